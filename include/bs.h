/*
 * bs.h -- C ABI of libbs.so: Ewald-split Biot-Savart velocity (and
 * streamfunction / energy) at the nodes of closed vortex filaments in a
 * triply periodic cubic box, on one AMD Instinct MI355X (gfx950).
 *
 * Paper: J. I. Polanco, "Fast and accurate evaluation of Biot-Savart
 * integrals over spatial curves in periodic domains", arXiv 2406.07366.
 *
 * Problem statement followed by the calls:
 *   - filaments are closed oriented curves given by ordered nodes
 *     (Sec. 2.1) carrying one circulation each (Sec. 2.2, eq:BS);
 *   - the curve through the nodes is the periodic cubic spline on
 *     chord-length knots (App. B); line integrals use Q Gauss-Legendre
 *     points per segment (Sec. 2.7, eq:line_integral_quadrature);
 *   - v = v_local + v_short + v_long - v_self (Sec. 3,
 *     eq:ewald_velocity_splitting), psi likewise
 *     (eq:ewald_streamfunction_splitting), with the local terms
 *     eq:BS_local / eq:streamfunction_local, the short-range sums
 *     eq:velocity_shortrange / eq:streamfunction_shortrange cut at r_c,
 *     the long-range part by a type-1 NUFFT, the Gaussian-filtered symbol
 *     i k x / k^2 (eq:velocity_longrange_physical) and a type-2 NUFFT
 *     (Sec. 3.3, App. A, backward Kaiser-Bessel kernel eq:kaiser_bessel_bw),
 *     and the self corrections eq:velocity_longrange_self /
 *     eq:streamfunction_longrange_self;
 *   - E = (1/2V) sum_l Gamma_l oint psi . ds
 *     (eq:kinetic_energy_streamfunction).
 *
 * Conventions shared by every call:
 *   - all floating-point arrays are float64; node arrays are [N][3]
 *     row-major (x, y, z of node 0, then node 1, ...);
 *   - "device" pointers are HIP device memory on the plan's device; the
 *     caller owns every array it passes; the plan owns its internal buffers;
 *   - calls are asynchronous on the plan's stream unless stated otherwise;
 *     results are ready once that stream has been synchronised;
 *   - return value: 0 (BS_OK) or a negative BS_E* code; bs_last_error()
 *     then holds a message.  A failed call leaves the plan usable.
 *   - one plan must not be used from two host threads at once.
 */
#ifndef BS_H
#define BS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BS_OK        0
#define BS_EINVAL   -1   /* bad argument, size, or filament geometry            */
#define BS_EMINIMG  -2   /* r_c > L/2: violates the minimum-image convention
                            (Sec. 5.2, footnote on r_c <= L/2)                 */
#define BS_ETOL     -3   /* tolerance unreachable on this grid (would need
                            r_c > L/2)                                        */
#define BS_EKB      -4   /* retained modes outside the kernel's band (|k|
                            scaled beyond the Kaiser-Bessel shape parameter)  */
#define BS_ENOMEM   -5   /* device allocation failed                          */
#define BS_EDEVICE  -6   /* HIP / hipFFT runtime error                        */
#define BS_ESTATE   -7   /* call out of order (e.g. velocity before filaments)*/

/* precision */
#define BS_FP64        0  /* every step in float64                            */
#define BS_FP32_MIXED  1  /* spread, FFT, interpolation and short-range pairs
                             in float32 with float32 accumulation; positions,
                             grid offsets and pair separations formed in
                             float64; local, self, k = 0 and reductions in
                             float64                                          */

/* near-singular treatment of (node, segment) pairs closer than
 * ns_eta * segment length (not part of the paper; see bs_velocity) */
#define BS_NS_OFF       0
#define BS_NS_ADAPTIVE  1  /* graded Gauss-Legendre panels on the spline segment
                              (relative error ~1e-11; the reference integrator) */
#define BS_NS_MLP       2  /* learned correction where its error indicator
                              allows, else the graded panels (bs_set_mlp)      */
#define BS_NS_MAPPED    3  /* fixed-cost rule: sinh-mapped 2 x 16-point
                              Gauss-Legendre split at the closest point, with
                              the tangent segment's closed form as a control
                              variate                                        */

/* 3-D transforms of the long-range step */
#define BS_FFT_AUTO     0  /* BS_FFT_PRUNED for power-of-two grids from 64 up
                              (where it is faster), else BS_FFT_LIBRARY         */
#define BS_FFT_LIBRARY  1  /* hipFFT: full r2c / c2r transforms and a separate
                              spectral-operator pass                           */
#define BS_FFT_PRUNED   2  /* grid_n a power of two (else BS_EINVAL): transforms
                              that form only the retained modes |m_i| <= K,
                              with the spectral operator fused into the z
                              transform                                        */

typedef struct bs_plan_s *bs_plan_t;

/* Parameters.  Zero in a derived field means "derive it":
 *   beta   from tol: the beta of the most accurate-enough row of the paper's
 *          Table 1 (tol 1e-3..1e-14 -> beta 2.0..5.5), i.e. the row with the
 *          largest tolerance <= tol;
 *   w      from tol: Table 1's width at the table's own tolerances (4, 6,
 *          8, ..., 16 for 1e-3, 1e-4, 1e-6, ..., 1e-14); at any other
 *          tolerance ceil(-log10(tol)/0.9) + 1 (NUFFT error ~10^(-0.9 w) at
 *          sigma = 1.5, App. A, Fig. accuracy_nufft), clamped to [4, 16];
 *   alpha  from the grid: M = floor(grid_n / sigma) resolved modes per
 *          axis, K = floor((M-1)/2), k_max = 2 pi K / L = 2 beta alpha
 *          (Sec. 4: k_max = 2 beta alpha, r_c = beta / alpha);
 *   rcut   = beta / alpha.
 * If alpha is given, rcut defaults to beta/alpha; if both are given they
 * are used as is. */
typedef struct {
    double L;            /* box period (cubic)                                 */
    double a;            /* vortex core radius                                 */
    double delta;        /* core-profile constant Delta (1/4: uniform core)    */
    double tol;          /* nominal relative tolerance                         */
    double beta;         /* cut-off coefficient (0: from tol)                  */
    double alpha;        /* Ewald splitting parameter (0: from grid and beta)  */
    double rcut;         /* short-range cut-off (0: beta/alpha)                */
    int    grid_n;       /* spread/FFT grid points per axis: a multiple of 4,
                            16..1024, at least w + 8 (w + 4 if not a multiple
                            of 8)                                           */
    double sigma;        /* oversampling factor (0: 1.5)                       */
    int    w;            /* kernel width in grid points (0: from tol)          */
    int    Q;            /* Gauss-Legendre points per segment, 1..4 (0: 2)     */
    int    spline_order; /* 4 = cubic, 6 = quintic (App. B; 0: 4)              */
    int    precision;    /* BS_FP64 or BS_FP32_MIXED                           */
    int    ns_mode;      /* BS_NS_OFF, BS_NS_ADAPTIVE, BS_NS_MLP or
                            BS_NS_MAPPED (the network is trained on cubic
                            segments: BS_NS_MLP needs spline_order 4; its
                            network is attached by bs_set_mlp)              */
    double ns_eta;       /* flag pairs with chord distance < ns_eta * ell (0: 1) */
    int    fft_mode;     /* BS_FFT_AUTO, BS_FFT_LIBRARY or BS_FFT_PRUNED; the
                            resolved parameters hold the choice made for
                            BS_FFT_AUTO                                     */
    double local_frac;   /* local-segment subdivision (Sec. 5.2): fraction of
                            each local segment, next to the node, where the
                            Taylor expansion of eq:BS_local and
                            eq:streamfunction_local is used; the rest of the
                            two local segments is integrated with the unsplit
                            kernels (3-point Gauss-Legendre on panels graded
                            towards the node).  0 or 1: whole segments      */
    /* resolved values, written by bs_resolve_params / bs_get_params */
    int    K;            /* retained modes |m_i| <= K per axis                 */
    int    ncell;        /* cells per axis of the short-range cell list (edge
                            >= 2 rcut / 3; 1 if fewer than 4 fit)            */
    double zeta;         /* Kaiser-Bessel shape parameter                      */
} bs_params;

/* Pure host call (no device needed): validate p and fill every derived
 * field into *out.  Errors: BS_EINVAL (L, a, tol, grid_n, sigma, w, Q,
 * spline_order out of range), BS_EMINIMG (rcut > L/2), BS_ETOL (derived
 * rcut would exceed L/2), BS_EKB. */
int bs_resolve_params(const bs_params *p, bs_params *out);

/* Create a plan on the current HIP device for one box period L, core a and
 * Delta (Sec. 2.3, eq:BS_local), Ewald parameters alpha, r_c (Sec. 3,
 * eq:ewald_velocity_splitting; Sec. 4 for beta) and NUFFT parameters sigma,
 * w (Sec. 3.3, App. A, Table 1), after bs_resolve_params' derivation.
 *   p           parameters (read during the call, not kept);
 *   hip_stream  a hipStream_t (NULL = the null stream); every later call
 *               enqueues on it;
 *   out         receives the handle (NULL on error).
 * Allocates the grids (3 [n]^3 reals and their spectra) and builds the FFT
 * plans; the plan owns them until bs_destroy.  Errors as
 * bs_resolve_params, plus BS_ENOMEM, BS_EDEVICE. */
int bs_plan(const bs_params *p, void *hip_stream, bs_plan_t *out);

/* Load a filament set: closed oriented curves through ordered nodes
 * (Sec. 2.1) with one circulation each (Sec. 2.2, eq:BS), interpolated by
 * the periodic spline on chord-length knots (App. B) and discretised by Q
 * Gauss-Legendre points per segment (Sec. 2.7,
 * eq:line_integral_quadrature).
 *   nfil     number of filaments (>= 1; closed unless bs_set_periods
 *            says otherwise);
 *   offsets  HOST int64 [nfil+1], offsets[0] = 0, filament l owns nodes
 *            offsets[l] .. offsets[l+1]-1, each filament has >= 3 nodes;
 *   xyz      DEVICE float64 [N][3], N = offsets[nfil], unwrapped positions
 *            (consecutive nodes close; the node after the last one is the
 *            first one at the same unwrapped position);
 *   gamma    DEVICE float64 [nfil], circulation of each filament.
 * The spline fit and quadrature geometry are computed here, asynchronously;
 * xyz and gamma are read before the call's work completes and are not kept.
 * Host-side errors: BS_EINVAL (sizes), BS_ENOMEM.  Non-finite positions or
 * zero-length segments are detected on the device and reported by the next
 * bs_status() (outputs computed from such input are meaningless). */
int bs_set_filaments(bs_plan_t plan, int64_t nfil, const int64_t *offsets,
                     const double *xyz, const double *gamma);

/* Infinite periodic filaments (Sec. 2.1: a curve that is not closed in the
 * cell but repeats with the domain, s(tau + T) = s(tau) + n L with n an
 * integer vector).
 *   nfil     number of filaments of the sets loaded afterwards;
 *   periods  HOST int64 [nfil][3]: n for each filament, (0,0,0) for a closed
 *            one; |n_i| <= 2^20.  NULL: every filament closed (the default).
 * For filament l with n != 0 the node after its last node is its first node
 * shifted by n L: the last segment, the spline (whose derivatives stay
 * periodic) and the local terms use that shifted node.  Positions are
 * otherwise as in bs_set_filaments (one period of nodes, unwrapped).  The
 * long-range sum omits k = 0 (eq:velocity_longrange_physical needs zero
 * mean vorticity): with sum_l Gamma_l n_l != 0 the result is that of the
 * filaments in a uniform background of the opposite mean vorticity.
 * The setting stays until changed; it drops the loaded filaments (and a
 * recorded bs_step graph), so bs_set_filaments must follow, with the same
 * nfil (BS_EINVAL otherwise).  Errors: BS_EINVAL (nfil < 1, |n_i| too
 * large), BS_ENOMEM; after an error every filament counts as closed.
 * Synchronises the plan stream. */
int bs_set_periods(bs_plan_t plan, int64_t nfil, const int64_t *periods);

/* Velocity at every node: v_out DEVICE float64 [N][3] (overwritten).
 * v = v_local + v_short + v_long - v_self (Sec. 3,
 * eq:ewald_velocity_splitting): the local term eq:BS_local, the short-range
 * sum eq:velocity_shortrange within r_c (minimum image), the long-range term
 * from the vorticity's Fourier coefficients eq:vorticity_fourier_coefs
 * through eq:velocity_longrange_physical (type-1 NUFFT, Gaussian-filtered
 * i k x / k^2, type-2 NUFFT; Sec. 3.3, App. A) and the self correction
 * eq:velocity_longrange_self.  Plus, when ns_mode is not BS_NS_OFF, the
 * near-singular correction (not in the paper): for every non-adjacent
 * segment whose chord lies closer than ns_eta * (segment length) to the
 * node, the Q-point sum of that segment is replaced by its integral of the
 * full Biot-Savart kernel (exact to rounding with BS_NS_ADAPTIVE; the mapped
 * rule's or the network's value with BS_NS_MAPPED, BS_NS_MLP).  At most 64 such segments per node are kept: a node
 * with more is reported by bs_status (BS_EINVAL).  BS_ESTATE if no
 * filaments were set (or BS_NS_MLP without bs_set_mlp).  The short-range
 * and near-singular terms run on a second stream that the plan owns, forked
 * from and joined back into the plan stream by events: as seen from the
 * plan stream, the call's work is ordered like any other. */
int bs_velocity(bs_plan_t plan, double *v_out);

/* Velocity split into its terms, each a DEVICE float64 [N][3] array or
 * NULL: local, short-range, long-range, self correction (to be subtracted)
 * and near-singular correction.  For tests and diagnostics. */
int bs_velocity_terms(bs_plan_t plan, double *v_local, double *v_short,
                      double *v_long, double *v_self, double *v_ns);

/* Streamfunction at every node (psi_out DEVICE [N][3], or NULL;
 * eq:ewald_streamfunction_splitting with eq:streamfunction_local,
 * eq:streamfunction_shortrange, the long-range streamfunction and
 * eq:streamfunction_longrange_self) and the kinetic energy per unit density
 * E = (1/2V) sum_l Gamma_l oint psi . ds (eq:kinetic_energy_streamfunction),
 * written to *E_out (HOST double, may be NULL); psi between the nodes is the
 * spline through its nodal values, integrated by the curve's Q-point rule.
 * Synchronises the plan stream.  BS_ESTATE if no filaments were set. */
int bs_energy(bs_plan_t plan, double *E_out, double *psi_out);

/* Fourier coefficients of the vorticity recovered from the spread grid
 * (type-1 NUFFT of the vector charges, eq:vorticity_fourier_coefs), for
 * the half space of modes: out DEVICE float64 complex as (re, im) pairs,
 * shape [K+1][2K+1][2K+1][3] indexed [mz][my+K][mx+K][component]; entries
 * outside the half space (mz = 0 and (my < 0 or my = 0 and mx <= 0)) are 0.
 * For tests of the spreading step. */
int bs_vorticity_modes(bs_plan_t plan, double *out);

/* Geometry of the loaded filaments, DEVICE float64 arrays or NULL:
 * quadrature point positions [N*Q][3] (unwrapped), vector charges
 * Gamma w_i dtau_j s'_ij [N*Q][3], node tangents ds/dtau [N][3], node
 * second derivatives d2s/dtau2 [N][3], segment lengths [N].  Point q =
 * j*Q + i lies on segment j (node j to its successor). */
int bs_geometry(bs_plan_t plan, double *qpos, double *qcharge, double *sdot,
                double *sddot, double *ell);

/* bs_set_filaments followed by bs_velocity.  With graph replay enabled
 * (bs_set_graph), the first call runs eagerly and then records the whole
 * sequence as a HIP graph; later calls with the same pointers and the same
 * offsets replay it with one launch.  If recording is not possible the plan
 * silently keeps running eagerly (bs_graph_active tells which). */
int bs_step(bs_plan_t plan, int64_t nfil, const int64_t *offsets, const double *xyz,
            const double *gamma, double *v_out);
/* enable (1) or disable (0) graph replay in bs_step; needs a non-null plan
 * stream (BS_EINVAL otherwise).  Disabled by default. */
int bs_set_graph(bs_plan_t plan, int enable);
/* 1 if bs_step currently replays a recorded graph */
int bs_graph_active(bs_plan_t plan);

/* One classical fourth-order Runge-Kutta step of dx/dt = v(x) for every
 * node (Sec. 5.2: each node moves with the Biot-Savart velocity; the spline
 * is refitted at every stage).  xyz: DEVICE float64 [N][3], advanced in
 * place; offsets (HOST) and gamma (DEVICE) as in bs_set_filaments; dt the
 * time step.  Leaves the plan loaded with the last stage's filaments. */
int bs_rk4_step(bs_plan_t plan, int64_t nfil, const int64_t *offsets, double *xyz,
                const double *gamma, double dt);

/* Synchronise the plan stream and report device-side input errors seen
 * since the last call (BS_EINVAL with a message), else BS_OK. */
int bs_status(bs_plan_t plan);

/* Per-stage timing, for measurement.  While enabled, bs_set_filaments and
 * bs_velocity record HIP events before and after each stage on the plan
 * stream and synchronise at their end, and bs_velocity runs its stages one
 * after another on the plan stream (otherwise the short-range sum and the
 * near-singular correction run on a second stream of the plan, beside the
 * long-range stages, joined before the call's work ends on the plan
 * stream); bs_stage_times returns the summed
 * milliseconds and the number of timed launches of each stage (arrays of
 * BS_NSTAGES, either may be NULL) and optionally resets them.  Stages:
 *   0 geometry (chord lengths, spline solve, quadrature points, and the
 *     velocity's local and self terms, all in one kernel)
 *   1 binning (counting sorts and sorted copies)
 *   2 (unused: the local and self terms are part of stage 0)
 *                               3 spread        4 forward FFT
 *   5 spectral operator         6 inverse FFT   7 interpolation
 *   8 short-range pairs         9 near-singular correction
 *  10 near-singular pair search (in bs_set_filaments, when ns_mode is on) */
#define BS_NSTAGES 11
int bs_set_profiling(bs_plan_t plan, int enable);
int bs_stage_times(bs_plan_t plan, double *ms, int64_t *counts, int reset);

/* ---- learned near-singular correction --------------------------------
 * A small network 8 -> 64 -> 64 -> 64 -> 3 with SiLU hidden activations,
 * BF16 weights on MFMA with FP32 accumulation (not part of the paper).
 * Parameters are FP32, packed W1[64][8] b1[64] W2[64][64] b2[64] W3[64][64]
 * b3[64] W4[3][64] b4[3] (bs_mlp_nparams() values, W row-major [out][in]).
 * X is float32 [B][8] (features), Y and T float32 [B][3], all DEVICE
 * pointers; calls are asynchronous on the stream given at creation. */
typedef struct bs_mlp_s *bs_mlp_t;
int bs_mlp_nparams(void);
/* copy params_host (FP32, bs_mlp_nparams() values) to the device; Adam
 * moments start at zero */
int bs_mlp_create(const float *params_host, void *hip_stream, bs_mlp_t *out);
/* Y = network(X) */
int bs_mlp_forward(bs_mlp_t m, int64_t B, const float *X, float *Y);
/* loss = (1/2B) sum |network(X) - T|^2 and its gradient w.r.t. the packed
 * parameters (loss_dev: 1 float, grad_dev: bs_mlp_nparams() floats; either
 * may be NULL) */
int bs_mlp_loss_grad(bs_mlp_t m, int64_t B, const float *X, const float *T,
                     float *loss_dev, float *grad_dev);
/* one Adam step on that loss (bias-corrected moments); loss_dev may be NULL */
int bs_mlp_adam_step(bs_mlp_t m, int64_t B, const float *X, const float *T,
                     float lr, float beta1, float beta2, float eps, float *loss_dev);
/* Debug mode (enable = 1): the forward, loss-gradient and Adam calls (and
 * the plans using this network) run the same kernels with FP32 weights and
 * activations on FP32 MFMA (v_mfma_f32_16x16x4_f32) instead of BF16, so that
 * their results differ from an FP64 evaluation by FP32 rounding only; for
 * checking the gradients.  enable = 0 returns to BF16. */
int bs_mlp_set_fp32(bs_mlp_t m, int enable);
/* synchronise and copy the current FP32 parameters to the host */
int bs_mlp_get_params(bs_mlp_t m, float *params_host);
int bs_mlp_destroy(bs_mlp_t m);

/* Training samples for the learned near-singular correction, generated on
 * the device by the plan's own graded Gauss-Legendre segment integrator
 * (float64).  U: DEVICE float64 [n][8] uniforms in [0,1) supplied by the
 * caller (they fix the segment tangents, the target's position class,
 * distance and azimuth); X: DEVICE float32 [n][8] features; T: DEVICE float32
 * [n][3] targets (I_seg - I_tan) / m in the chord frame (chord length h = 1),
 * I_tan the straight segment tangent to the curve at its point closest to
 * the target, d that distance and m = 1 + log(1 + h/d); aux: DEVICE float64
 * [n][7] (d/h, exact raw integral (3), m, the tangent segment's absolute
 * integral S = int |ds|/|s-x|^2 that errors are measured against, chord
 * distance / h) or NULL.  The
 * sample box: tangent angles <= 0.6 rad, tangent lengths in [0.9, 1.1],
 * d_c/h log-uniform in bs_ns_error_bins' range. */
int bs_ns_samples(int64_t n, const double *U, float *X, float *T, double *aux,
                  void *hip_stream);
/* range [lo, hi] of (distance to the chord)/h covered by the network, and
 * the number of log-spaced bins of its error table (binned by the distance
 * to the chord over h, values outside [lo, hi] falling in the end bins) */
int bs_ns_error_bins(double *lo, double *hi, int *nbins);
/* Error table of a trained network on held-out samples of bs_ns_samples
 * (X, T DEVICE float32 [n][8], [n][3]; aux DEVICE float64 [n][7], as
 * written by bs_ns_samples; n >= 1): per distance bin (bs_ns_error_bins),
 * the root-mean-square (rms_out) and largest (max_out) error of the learned
 * raw segment integral |I_tan + m y - I| in units of the chord length
 * (h = 1), I the plain method's graded-panel integral; HOST float [nbins]
 * each (either may be NULL); +inf in a bin without samples.  Runs on the
 * network's stream and synchronises it; allocates and frees a scratch of
 * 12 n bytes.  Errors: BS_EINVAL (sizes, nbins), BS_ENOMEM, BS_EDEVICE. */
int bs_ns_error_table(bs_mlp_t mlp, int64_t n, const float *X, const float *T,
                      const double *aux, float *rms_out, float *max_out, int nbins);
/* bs_ns_error_table for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same table, written to rms_out and max_out as DEVICE float [nbins]
 * arrays (either may be NULL), asynchronously on the network's stream (no
 * host copy, no synchronisation).  Calls no hipMalloc, hipFree or other
 * allocating routine: the network outputs and partial sums live in a
 * static device array of 3.2 MB per GPU, held until the process ends, so n
 * is at most 262144 (BS_EINVAL beyond).  Calls on one GPU share that array:
 * calls that overlap on one GPU (two streams, two threads) race.  Errors:
 * BS_EINVAL (sizes, nbins), BS_EDEVICE. */
int bs_ns_error_table_noalloc(bs_mlp_t mlp, int64_t n, const float *X, const float *T,
                              const double *aux, float *rms_out, float *max_out, int nbins);
/* Attach a trained network to a BS_NS_MLP plan.  err_table[nbins] holds the
 * rms error per distance bin (bs_ns_error_table's rms_out).  A pair (node
 * i, segment of length h, circulation Gamma) takes the learned integral
 * when its inputs lie in the sample box and
 *     err_table[bin] * |Gamma| / (4 pi h) * sqrt(P / N) <= tol * v_scale,
 * P the flagged pairs of the N nodes and v_scale the rms over the nodes of
 * the velocity's local, self and short-range terms (formed before the
 * correction): the pairs' errors then add to at most about tol times the rms
 * velocity.  Every other pair takes the graded panels (BS_NS_ADAPTIVE).  The
 * table is copied; the plan keeps the network handle, which must outlive
 * its use by the plan.  Drops a recorded bs_step graph.  Errors: BS_ESTATE
 * (plan not BS_NS_MLP), BS_EINVAL (null network, nbins, negative entry). */
int bs_set_mlp(bs_plan_t plan, bs_mlp_t mlp, const float *err_table, int nbins);
/* Synchronise; number of flagged near-singular pairs of the loaded
 * filaments, and number of those the learned path handed to the graded
 * panels in the last velocity evaluation (0 if none ran; the network carried
 * the rest). */
int bs_ns_counts(bs_plan_t plan, int64_t *npairs, int64_t *nfallback);

/* Parameters actually used (all derived fields filled). */
int bs_get_params(bs_plan_t plan, bs_params *resolved);

/* Release every device buffer and FFT plan; synchronises first. */
int bs_destroy(bs_plan_t plan);

/* Message of the last failed call on this plan (or of the last failed
 * bs_plan / bs_resolve_params when plan is NULL).  Never NULL. */
const char *bs_last_error(bs_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* BS_H */
