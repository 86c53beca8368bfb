// C ABI of libbs.so: parameter resolution, plan and buffer management, and
// the order of the steps of one velocity / energy evaluation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "bs_internal.h"

namespace bs {

static thread_local std::string g_err = "no error";

int set_error(bs_plan_t p, int code, const std::string &msg) {
    if (p) p->err = msg;
    else g_err = msg;
    return code;
}

int check_hip(bs_plan_t p, hipError_t e, const char *what) {
    if (e == hipSuccess) return BS_OK;
    return set_error(p, e == hipErrorOutOfMemory ? BS_ENOMEM : BS_EDEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

// Gauss-Legendre rule on [-1, 1] by Newton iteration on the three-term
// recurrence of the Legendre polynomials; nodes ascending.
static void legendre_rule(int n, double *x, double *w) {
    for (int i = 0; i < n; i++) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

GLRule gl_rule(int Q) {
    GLRule r{};
    double x[kMaxQ], w[kMaxQ];
    if (Q == 1) { x[0] = 0.0; w[0] = 2.0; }
    else legendre_rule(Q, x, w);
    for (int i = 0; i < Q; i++) { r.h[i] = 0.5 * (x[i] + 1.0); r.w[i] = 0.5 * w[i]; }
    return r;
}

// Host copy of the normalised kernel phi(z) = sinh(zeta s)/(sinh(zeta) s),
// s = sqrt(1 - z^2) (same normalisation as the device kernel).
static double kb_phi_host(double z, double zeta) {
    double s2 = 1.0 - z * z;
    double den = -std::expm1(-2.0 * zeta);
    if (s2 <= 0.0) return 2.0 * zeta * std::exp(-zeta) / den;
    double s = std::sqrt(s2);
    return std::exp(zeta * (s - 1.0)) * (-std::expm1(-2.0 * zeta * s)) / s / den;
}

// F(m) = (w/2) int_{-1}^{1} phi(z) cos(pi m w z / n) dz, the transform of the
// spreading kernel per axis (Poisson summation of the grid sum; App. A).
// The integrand is analytic on [-1,1], so a 256-point Gauss-Legendre rule is
// exact to rounding.  (The closed form I0(sqrt(zeta^2 - kappa^2)) of
// eq:kaiser_bessel_bw is the transform of the kernel continued beyond
// |z| = 1 and differs from the truncated kernel's by ~e^{-zeta}.)
static void kernel_ft_table(int K, int w, int n, double zeta, double *F) {
    const int nq = 256;
    std::vector<double> x(nq), wt(nq), ph(nq);
    legendre_rule(nq, x.data(), wt.data());
    for (int i = 0; i < nq; i++) ph[i] = kb_phi_host(x[i], zeta);
    for (int m = 0; m <= K; m++) {
        double kap = kPi * m * w / n, s = 0.0;
        for (int i = 0; i < nq; i++) s += wt[i] * ph[i] * std::cos(kap * x[i]);
        F[m] = 0.5 * w * s;
    }
}

// Gauss-Legendre rules of the near-singular integrals: 16 points (the mapped
// rule, each side of the peak), 10 and 12 points (the graded panels on cubic
// and quintic segments)
struct NsRule {
    double x[16], w[16];
    double x10[10], w10[10];
    double x12[12], w12[12];
};
void ns_rule(NsRule *R) {
    static const NsRule cached = [] {
        NsRule r;
        legendre_rule(16, r.x, r.w);
        legendre_rule(10, r.x10, r.w10);
        legendre_rule(12, r.x12, r.w12);
        return r;
    }();
    *R = cached;
}

template <typename T>
static int ensure(bs_plan_t p, DBuf &b, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (b.bytes >= bytes) return BS_OK;
    if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) { b.p = nullptr; return check_hip(p, e, "hipMalloc"); }
    b.bytes = bytes;
    return BS_OK;
}

static void release(DBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

__global__ void k_fill_f64(double *p, size_t n, double v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static void fill_f64(bs_plan_t p, double *ptr, size_t n, double v) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, ptr,
                       n, v);
}

__global__ void k_add_f64(double *__restrict__ y, const double *__restrict__ x, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i];
}

static void add_f64(bs_plan_t p, double *y, const double *x, size_t n) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_add_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, y, x,
                       n);
}

static int launch_status(bs_plan_t p, const char *what) {
    return check_hip(p, hipGetLastError(), what);
}

// Table 1 of the paper: nominal tolerance -> beta and kernel width w.
static const double kTabTol[7] = {1e-3, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14};
static const double kTabBeta[7] = {2.0, 2.5, 3.5, 4.0, 4.5, 5.0, 5.5};
static const int kTabW[7] = {4, 6, 8, 10, 12, 14, 16};

static double beta_from_tol(double tol) {
    for (int i = 0; i < 7; i++)
        if (kTabTol[i] <= tol * (1.0 + 1e-9)) return kTabBeta[i];
    return kTabBeta[6];
}

// a tolerance of the table takes the table's width; any other the App. A
// decay law 10^(-0.9 w)
static int width_from_tol(double tol) {
    for (int i = 0; i < 7; i++)
        if (std::fabs(tol - kTabTol[i]) <= 1e-9 * kTabTol[i]) return kTabW[i];
    double pe = -std::log10(tol);
    int w = (int)std::ceil(pe / 0.9 - 1e-9) + 1;
    return std::min(kMaxW, std::max(kMinW, w));
}

int resolve(const bs_params *in, bs_params *out) {
    if (!in || !out) return set_error(nullptr, BS_EINVAL, "null parameter pointer");
    bs_params r = *in;
    auto bad = [](const char *m) { return set_error(nullptr, BS_EINVAL, m); };
    if (!(std::isfinite(r.L) && r.L > 0)) return bad("L must be positive");
    if (!(std::isfinite(r.a) && r.a > 0 && r.a < r.L)) return bad("a must be in (0, L)");
    if (!std::isfinite(r.delta)) return bad("delta must be finite");
    if (!(r.tol > 0 && r.tol <= 0.5)) return bad("tol must be in (0, 0.5]");
    if (r.grid_n < 16 || r.grid_n % 4 != 0 || r.grid_n > 1024)
        return bad("grid_n must be a multiple of 4 in [16, 1024]");
    if (r.sigma == 0) r.sigma = 1.5;
    if (!(r.sigma > 1.0 && r.sigma <= 4.0)) return bad("sigma must be in (1, 4]");
    if (r.Q == 0) r.Q = 2;
    if (r.Q < 1 || r.Q > kMaxQ) return bad("Q must be in 1..4");
    if (r.spline_order == 0) r.spline_order = 4;
    if (r.spline_order != 4 && r.spline_order != 6)
        return bad("spline_order must be 4 (cubic) or 6 (quintic)");
    if (!(r.local_frac >= 0.0 && r.local_frac <= 1.0)) return bad("local_frac must be in [0, 1]");
    if (r.local_frac > 0.0 && r.local_frac < 1e-3)
        return bad("local_frac below 1e-3 (more than 10 panels per local segment)");
    if (r.precision != BS_FP64 && r.precision != BS_FP32_MIXED) return bad("unknown precision");
    if (r.ns_mode < BS_NS_OFF || r.ns_mode > BS_NS_MAPPED) return bad("unknown ns_mode");
    if (r.ns_mode == BS_NS_MLP && r.spline_order != 4)
        return bad("the learned near-singular correction is trained on cubic segments only");
    if (r.ns_eta == 0) r.ns_eta = 1.0;
    if (!(r.ns_eta > 0)) return bad("ns_eta must be positive");
    if (r.fft_mode < BS_FFT_AUTO || r.fft_mode > BS_FFT_PRUNED) return bad("unknown fft_mode");
    {
        const bool ok = pruned_fft_ok(r.grid_n, r.precision == BS_FP32_MIXED ? 8 : 16);
        if (r.fft_mode == BS_FFT_PRUNED && !ok)
            return bad("BS_FFT_PRUNED needs grid_n a power of two (at most 512 in float64)");
        // automatic choice: the pruned transforms win from 64^3 up (measured);
        // hipFFT on smaller grids
        if (r.fft_mode == BS_FFT_AUTO)
            r.fft_mode = (ok && r.grid_n >= 64) ? BS_FFT_PRUNED : BS_FFT_LIBRARY;
    }
    if (r.beta == 0) r.beta = beta_from_tol(r.tol);
    if (!(r.beta > 0)) return bad("beta must be positive");
    if (r.w == 0) r.w = width_from_tol(r.tol);
    if (r.w < kMinW || r.w > kMaxW) return bad("w must be in 4..16");
    {
        // every stencil must reach a spread tile at most once along an axis
        int T = (r.grid_n % 8 == 0) ? 8 : 4;
        if (r.grid_n < r.w + T) return bad("grid_n must be at least w + 8 (w + 4 if not a multiple of 8)");
    }
    int M = (int)std::floor(r.grid_n / r.sigma + 1e-9);
    r.K = (M - 1) / 2;
    if (r.K < 1) return bad("grid too small for one retained mode");
    bool derived = (in->alpha == 0 && in->rcut == 0);
    if (r.alpha == 0) r.alpha = r.K * (2.0 * kPi / r.L) / (2.0 * r.beta);
    if (!(r.alpha > 0)) return bad("alpha must be positive");
    if (r.rcut == 0) r.rcut = r.beta / r.alpha;
    if (!(r.rcut > 0)) return bad("rcut must be positive");
    if (r.rcut > 0.5 * r.L * (1.0 + 1e-12)) {
        if (derived)
            return set_error(nullptr, BS_ETOL,
                             "tolerance needs r_c = beta/alpha > L/2 on this grid; use a larger "
                             "grid_n");
        return set_error(nullptr, BS_EMINIMG, "rcut > L/2 violates the minimum-image convention");
    }
    r.zeta = 0.995 * r.w * kPi * (1.0 - 1.0 / (2.0 * r.sigma));
    double kap_max = kPi * r.K * r.w / r.grid_n;
    if (kap_max >= r.zeta)
        return set_error(nullptr, BS_EKB, "retained modes beyond the kernel's band (raise sigma)");
    // short-range cells of edge >= 2 r_c / 3: the points within r_c of any
    // target lie in a 4 x 4 x 4 block of cells (one cell when fewer than 4
    // fit along an axis)
    int nc = (int)std::floor(3.0 * r.L / (2.0 * r.rcut * (1.0 + 1e-6)));
    if (nc < 4) nc = 1;
    if (nc > 160) nc = 160;
    r.ncell = nc;
    *out = r;
    return BS_OK;
}

void stage_collect(bs_plan_t p) {
    if (!p->prof) return;
    (void)hipStreamSynchronize(p->stream);
    for (int s = 0; s < BS_NSTAGES; s++) {
        if (!p->ev_used[s]) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p->ev_beg[s], p->ev_end[s]) == hipSuccess) {
            p->stage_ms[s] += ms;
            p->stage_cnt[s] += 1;
        }
        p->ev_used[s] = false;
    }
}

}  // namespace bs

using namespace bs;

extern "C" {

int bs_set_profiling(bs_plan_t P, int enable) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (enable && !P->ev_beg[0]) {
        for (int s = 0; s < BS_NSTAGES; s++) {
            int rc = check_hip(P, hipEventCreate(&P->ev_beg[s]), "hipEventCreate");
            if (!rc) rc = check_hip(P, hipEventCreate(&P->ev_end[s]), "hipEventCreate");
            if (rc) return rc;
        }
    }
    P->prof = enable != 0;
    return BS_OK;
}

int bs_stage_times(bs_plan_t P, double *ms, int64_t *counts, int reset) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    for (int s = 0; s < BS_NSTAGES; s++) {
        if (ms) ms[s] = P->stage_ms[s];
        if (counts) counts[s] = P->stage_cnt[s];
        if (reset) { P->stage_ms[s] = 0.0; P->stage_cnt[s] = 0; }
    }
    return BS_OK;
}

int bs_resolve_params(const bs_params *p, bs_params *out) { return resolve(p, out); }

const char *bs_last_error(bs_plan_t plan) { return plan ? plan->err.c_str() : g_err.c_str(); }

int bs_plan(const bs_params *p, void *hip_stream, bs_plan_t *out) {
    if (!out) return set_error(nullptr, BS_EINVAL, "null output handle");
    *out = nullptr;
    bs_params r;
    int rc = resolve(p, &r);
    if (rc) return rc;
    bs_plan_t P = new bs_plan_s();
    P->prm = r;
    P->stream = (hipStream_t)hip_stream;
    P->fp32 = (r.precision == BS_FP32_MIXED);
    P->real_size = P->fp32 ? 4 : 8;
    P->n = r.grid_n;
    P->T = (P->n % 8 == 0) ? 8 : 4;
    P->NT = P->n / P->T;
    P->nc = r.ncell;
    P->Q = r.Q;
    P->order = r.spline_order;
    (void)hipGetDevice(&P->device);
    const size_t n = (size_t)P->n, n3 = n * n * n, nc = n * n * (n / 2 + 1);
    auto fail = [&](int code) {
        g_err = P->err;
        bs_destroy(P);
        return code;
    };
    if ((rc = check_hip(P, hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking),
                        "hipStreamCreateWithFlags")) ||
        (rc = check_hip(P, hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming),
                        "hipEventCreateWithFlags")) ||
        (rc = check_hip(P, hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming),
                        "hipEventCreateWithFlags")) ||
        (rc = check_hip(P, hipEventCreateWithFlags(&P->ev_ns, hipEventDisableTiming),
                        "hipEventCreateWithFlags")))
        return fail(rc);
    if ((rc = ensure<char>(P, P->grid, 3 * n3 * P->real_size))) return fail(rc);
    if ((rc = ensure<char>(P, P->spec, 3 * nc * 2 * P->real_size))) return fail(rc);
    if ((rc = ensure<double>(P, P->deconv, 2 * (r.K + 1)))) return fail(rc);
    if ((rc = ensure<int>(P, P->d_status, 1))) return fail(rc);
    if ((rc = ensure<int>(P, P->red_tmp, 8192))) return fail(rc);
    if ((rc = ensure<int>(P, P->scan_tmp, 8192))) return fail(rc);
    if ((rc = check_hip(P, hipMemsetAsync(P->d_status.p, 0, sizeof(int), P->stream), "memset")))
        return fail(rc);
    // deconvolution table: [1/F(m)] then [1/F(m)^2], m = 0..K
    std::vector<double> F(r.K + 1), tab(2 * (r.K + 1));
    kernel_ft_table(r.K, r.w, P->n, r.zeta, F.data());
    for (int m = 0; m <= r.K; m++) {
        tab[m] = 1.0 / F[m];
        tab[r.K + 1 + m] = 1.0 / (F[m] * F[m]);
    }
    if ((rc = check_hip(P, hipMemcpy(P->deconv.p, tab.data(), tab.size() * sizeof(double),
                                     hipMemcpyHostToDevice), "copy table")))
        return fail(rc);
    // FFT plans: 3 transforms of n^3 (real) <-> n^2 (n/2+1) (complex)
    int dims[3] = {P->n, P->n, P->n};
    size_t ws = 0;
    if (hipfftCreate(&P->fft_fwd) != HIPFFT_SUCCESS || hipfftCreate(&P->fft_inv) != HIPFFT_SUCCESS)
        return fail(set_error(P, BS_EDEVICE, "hipfftCreate failed"));
    hipfftType tf = P->fp32 ? HIPFFT_R2C : HIPFFT_D2Z, ti = P->fp32 ? HIPFFT_C2R : HIPFFT_Z2D;
    if (hipfftMakePlanMany(P->fft_fwd, 3, dims, nullptr, 1, (int)n3, nullptr, 1, (int)nc, tf, 3,
                           &ws) != HIPFFT_SUCCESS ||
        hipfftMakePlanMany(P->fft_inv, 3, dims, nullptr, 1, (int)nc, nullptr, 1, (int)n3, ti, 3,
                           &ws) != HIPFFT_SUCCESS)
        return fail(set_error(P, BS_EDEVICE, "hipfftMakePlanMany failed"));
    if (hipfftSetStream(P->fft_fwd, P->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(P->fft_inv, P->stream) != HIPFFT_SUCCESS)
        return fail(set_error(P, BS_EDEVICE, "hipfftSetStream failed"));
    // pruned transforms: twiddles exp(-+2 pi i k / n), k < n/2, from float64
    P->pruned = r.fft_mode == BS_FFT_PRUNED;   // resolved: never BS_FFT_AUTO here
    if (P->pruned) {
        const size_t cs = 2 * P->real_size, K1 = r.K + 1, NY = 2 * r.K + 1;
        pruned_batches(P->n, cs, &P->fft_rb, &P->fft_kb, &P->fft_kz);
        if ((rc = ensure<char>(P, P->fft_tw, 2 * n * cs)) ||
            (rc = ensure<char>(P, P->fft_A, 3 * n * n * K1 * cs)) ||
            (rc = ensure<char>(P, P->fft_B, 3 * NY * n * K1 * cs)))
            return fail(rc);
        // [n] exp(-2 pi i k / n), then [n] exp(+2 pi i k / n)
        std::vector<double> tw(4 * n);
        for (size_t k = 0; k < n; k++) {
            const double ang = 2.0 * kPi * (double)k / (double)n;
            const double c = cos(ang), sn = sin(ang);
            tw[2 * k] = c; tw[2 * k + 1] = -sn;
            tw[2 * n + 2 * k] = c; tw[2 * n + 2 * k + 1] = sn;
        }
        if (P->fp32) {
            std::vector<float> tf(tw.begin(), tw.end());
            rc = check_hip(P, hipMemcpy(P->fft_tw.p, tf.data(), tf.size() * 4,
                                        hipMemcpyHostToDevice), "copy twiddles");
        } else {
            rc = check_hip(P, hipMemcpy(P->fft_tw.p, tw.data(), tw.size() * 8,
                                        hipMemcpyHostToDevice), "copy twiddles");
        }
        if (rc) return fail(rc);
    }
    *out = P;
    return BS_OK;
}

static void drop_graph(bs_plan_t P);

// order the plan stream after the side stream's pending pair search (the
// calls that read its results or overwrite its inputs on the plan stream)
static int join_side(bs_plan_t P) {
    if (!P->side_pending) return BS_OK;
    int rc = check_hip(P, hipStreamWaitEvent(P->stream, P->ev_ns, 0), "hipStreamWaitEvent");
    if (!rc) P->side_pending = false;
    return rc;
}

int bs_set_periods(bs_plan_t P, int64_t nfil, const int64_t *periods) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    drop_graph(P);
    P->have_filaments = false;
    P->nper = 0;
    if (!periods) return BS_OK;
    if (nfil < 1) return set_error(P, BS_EINVAL, "need nfil >= 1");
    std::vector<double> sh(3 * nfil);
    bool any = false;
    for (int64_t k = 0; k < 3 * nfil; k++) {
        if (periods[k] < -(1 << 20) || periods[k] > (1 << 20))
            return set_error(P, BS_EINVAL, "period counts must lie in [-2^20, 2^20]");
        sh[k] = (double)periods[k] * P->prm.L;
        any = any || periods[k] != 0;
    }
    if (!any) return BS_OK;   // all closed
    int rc;
    if ((rc = ensure<double>(P, P->d_shift, 3 * nfil)) ||
        (rc = check_hip(P, hipMemcpyAsync(P->d_shift.p, sh.data(), sizeof(double) * 3 * nfil,
                                          hipMemcpyHostToDevice, P->stream), "copy shifts")) ||
        (rc = check_hip(P, hipStreamSynchronize(P->stream), "sync")))
        return rc;
    P->nper = nfil;
    return BS_OK;
}

int bs_set_filaments(bs_plan_t P, int64_t nfil, const int64_t *offsets, const double *xyz,
                     const double *gamma) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (nfil < 1 || !offsets || !xyz || !gamma)
        return set_error(P, BS_EINVAL, "need nfil >= 1 and non-null offsets, xyz, gamma");
    if (offsets[0] != 0) return set_error(P, BS_EINVAL, "offsets[0] must be 0");
    int64_t maxn = 0;
    for (int64_t f = 0; f < nfil; f++) {
        int64_t c = offsets[f + 1] - offsets[f];
        if (c < 3) return set_error(P, BS_EINVAL, "every filament needs at least 3 nodes");
        if (P->order == 6 && c < 6)
            return set_error(P, BS_EINVAL, "quintic splines need at least 6 nodes per filament");
        maxn = std::max(maxn, c);
    }
    const int64_t N = offsets[nfil], Nq = N * P->Q;
    if (Nq >= ((int64_t)1 << 31) / 4) return set_error(P, BS_EINVAL, "too many nodes");
    int rc0 = join_side(P);   // the previous search reads what this call rewrites
    if (rc0) return rc0;
    if (P->nper && P->nper != nfil)
        return set_error(P, BS_EINVAL, "periods were set for " + std::to_string(P->nper) +
                                           " filaments, not " + std::to_string(nfil));
    bool same = P->have_filaments && P->nfil == nfil &&
                std::equal(offsets, offsets + nfil + 1, P->off_host.begin());
    int rc;
    const int ntiles = P->NT * P->NT * P->NT, nc3 = P->nc * P->nc * P->nc;
    const size_t rs = P->real_size;
    if (!same) {
        P->have_filaments = false;
        if ((rc = ensure<int>(P, P->d_off, nfil + 1)) || (rc = ensure<int>(P, P->d_fil, N)) ||
            (rc = ensure<double>(P, P->d_gamma, nfil)) || (rc = ensure<double>(P, P->d_x, 3 * N)) ||
            (rc = ensure<double>(P, P->d_xn, 3 * N)) ||
            (rc = ensure<double>(P, P->d_dtau, N)) || (rc = ensure<double>(P, P->d_D, 3 * N)) ||
            (rc = ensure<double>(P, P->d_sdd, 3 * N)) || (rc = ensure<double>(P, P->d_ell, N)) ||
            (rc = ensure<double>(P, P->d_qpos, 3 * Nq)) ||
            (rc = ensure<double>(P, P->d_qchg, 3 * Nq)) || (rc = ensure<double>(P, P->tmp3, 3 * N)) ||
            (rc = ensure<double>(P, P->e_D, 3 * N)) || (rc = ensure<double>(P, P->e_S, 3 * N)) ||
            (rc = ensure<double>(P, P->d_vls, 3 * N)) ||
            (rc = ensure<int>(P, P->sp_key, Nq)) || (rc = ensure<int>(P, P->sp_cnt, ntiles + 1)) ||
            (rc = ensure<int>(P, P->sp_start, ntiles + 1)) ||
            (rc = ensure<int>(P, P->sp_fill, ntiles + 1)) || (rc = ensure<int>(P, P->sp_perm, Nq)) ||
            (rc = ensure<int4>(P, P->sp_base, Nq)) ||
            (rc = ensure<char>(P, P->sp_ker, Nq * 3 * P->prm.w * rs)) ||
            (rc = ensure<char>(P, P->sp_q, Nq * 4 * rs)) || (rc = ensure<int>(P, P->pq_key, Nq)) ||
            (rc = ensure<int>(P, P->pq_cnt, nc3 + 1)) || (rc = ensure<int>(P, P->pq_start, nc3 + 1)) ||
            (rc = ensure<int>(P, P->pq_fill, nc3 + 1)) || (rc = ensure<int>(P, P->pq_perm, Nq)) ||
            (rc = ensure<double4>(P, P->pq_pos, Nq)) || (rc = ensure<char>(P, P->pq_chg, Nq * 4 * rs)) ||
            (rc = ensure<int>(P, P->nd_key, N)) ||
            (rc = ensure<int>(P, P->nd_cnt, nc3 + 1)) || (rc = ensure<int>(P, P->nd_start, nc3 + 1)) ||
            (rc = ensure<int>(P, P->nd_fill, nc3 + 1)) || (rc = ensure<int>(P, P->nd_perm, N)))
            return rc;
        if (P->order == 4 && maxn > kPcrLds && (rc = ensure<double>(P, P->spline_tmp, 12 * N)))
            return rc;
        if (P->order == 6 && maxn > kPcr5Lds &&
            (rc = ensure<double>(P, P->spline_tmp, 36 * N)))
            return rc;
        if (P->prm.ns_mode != BS_NS_OFF) {
            size_t mp = (size_t)N * P->ns_max_per_node;
            int ncmax = (int)cbrt(2.0 * (double)N);
            P->ns_ncmax = ncmax < 3 ? 3 : (ncmax > 128 ? 128 : ncmax);
            const size_t nb3 = (size_t)P->ns_ncmax * P->ns_ncmax * P->ns_ncmax;
            if ((rc = ensure<double>(P, P->ns_red, 2 * 1024 + 1)) ||
                (rc = ensure<int>(P, P->ns_nc, 2)) || (rc = ensure<int>(P, P->ns_ckey, N)) ||
                (rc = ensure<int>(P, P->ns_ccnt, 2 * nb3 + 1)) ||
                (rc = ensure<int>(P, P->ns_cstart, 2 * nb3 + 1)) ||
                (rc = ensure<int>(P, P->ns_cfill, 2 * nb3 + 1)) || (rc = ensure<int>(P, P->ns_cperm, N)) ||
                (rc = ensure<int>(P, P->ns_tkey, N)) || (rc = ensure<int>(P, P->ns_tcnt, nb3 + 1)) ||
                (rc = ensure<int>(P, P->ns_tstart, nb3 + 1)) ||
                (rc = ensure<int>(P, P->ns_tfill, nb3 + 1)) || (rc = ensure<int>(P, P->ns_tperm, N)) ||
                (rc = ensure<double4>(P, P->ns_segA, N)) || (rc = ensure<double4>(P, P->ns_segB, N)) ||
                (rc = ensure<float4>(P, P->ns_segM, N)) ||
                (rc = ensure<float4>(P, P->ns_segH, N)) ||
                (rc = ensure<int2>(P, P->ns_slots, mp)) || (rc = ensure<int>(P, P->ns_cnt, N + 1)) ||
                (rc = ensure<int>(P, P->ns_start, N + 1)) || (rc = ensure<int2>(P, P->ns_pairs, mp)) ||
                (rc = ensure<int>(P, P->ns_pnode, mp)) || (rc = ensure<double>(P, P->ns_pout, 3 * mp)))
                return rc;
            if (P->prm.ns_mode == BS_NS_MLP &&
                ((rc = ensure<float>(P, P->ns_X, 8 * mp)) || (rc = ensure<float>(P, P->ns_Y, 3 * mp)) ||
                 (rc = ensure<int>(P, P->ns_fallback, 4)) || (rc = ensure<int>(P, P->ns_learn, mp)) ||
                 (rc = ensure<int>(P, P->ns_fblist, mp)) || (rc = ensure<double>(P, P->ns_vs, 1 + 3 * 256))))
                return rc;
        }
        // the bin counters start at zero; afterwards each call's per-bin
        // sort clears them for the next
        const size_t nb_t = sizeof(int) * (ntiles + 1), nb_c = sizeof(int) * (nc3 + 1);
        if ((rc = check_hip(P, hipMemsetAsync(P->sp_cnt.p, 0, nb_t, P->stream), "memset")) ||
            (rc = check_hip(P, hipMemsetAsync(P->sp_fill.p, 0, nb_t, P->stream), "memset")) ||
            (rc = check_hip(P, hipMemsetAsync(P->pq_cnt.p, 0, nb_c, P->stream), "memset")) ||
            (rc = check_hip(P, hipMemsetAsync(P->pq_fill.p, 0, nb_c, P->stream), "memset")) ||
            (rc = check_hip(P, hipMemsetAsync(P->nd_cnt.p, 0, nb_c, P->stream), "memset")) ||
            (rc = check_hip(P, hipMemsetAsync(P->nd_fill.p, 0, nb_c, P->stream), "memset")) ||
            (P->ns_fallback.p &&
             (rc = check_hip(P, hipMemsetAsync(P->ns_fallback.p, 0, P->ns_fallback.bytes,
                                               P->stream), "memset"))))
            return rc;
        std::vector<int> off32(nfil + 1), fil32(N);
        for (int64_t f = 0; f <= nfil; f++) off32[f] = (int)offsets[f];
        for (int64_t f = 0; f < nfil; f++)
            for (int64_t j = offsets[f]; j < offsets[f + 1]; j++) fil32[j] = (int)f;
        if ((rc = check_hip(P, hipMemcpyAsync(P->d_off.p, off32.data(), sizeof(int) * (nfil + 1),
                                              hipMemcpyHostToDevice, P->stream), "copy offsets")) ||
            (rc = check_hip(P, hipMemcpyAsync(P->d_fil.p, fil32.data(), sizeof(int) * N,
                                              hipMemcpyHostToDevice, P->stream), "copy fil")))
            return rc;
        // the host vectors die at return: wait for the copies
        if ((rc = check_hip(P, hipStreamSynchronize(P->stream), "sync"))) return rc;
        P->off_host.assign(offsets, offsets + nfil + 1);
        P->nfil = nfil;
        P->N = N;
        P->Nq = Nq;
        P->max_fil_nodes = maxn;
    }
    stage_begin(P, 0);
    launch_filaments(P, xyz, gamma);   // also takes the plan's copies of xyz and gamma
    stage_end(P, 0);
    if (P->prm.ns_mode != BS_NS_OFF) {
        // the pair search needs only the geometry: it runs on the side stream,
        // beside the binning, and the velocity's short-range and
        // near-singular terms follow it there (per-stage timing keeps it on
        // the plan's stream)
        const bool side = !P->prof;
        if (side &&
            ((rc = check_hip(P, hipEventRecord(P->ev_fork, P->stream), "hipEventRecord")) ||
             (rc = check_hip(P, hipStreamWaitEvent(P->side, P->ev_fork, 0), "hipStreamWaitEvent"))))
            return rc;
        const hipStream_t plan_stream = P->stream;
        if (side) P->stream = P->side;
        stage_begin(P, 10);
        ns_build_pairs(P);
        stage_end(P, 10);
        P->stream = plan_stream;
        if (side) {
            if ((rc = check_hip(P, hipEventRecord(P->ev_ns, P->side), "hipEventRecord"))) return rc;
            P->side_pending = true;
        }
    }
    stage_begin(P, 1);
    build_bins(P);
    stage_end(P, 1);
    if ((rc = launch_status(P, "geometry kernels"))) return rc;
    P->have_filaments = true;
    stage_collect(P);
    return BS_OK;
}

// out += near-singular correction; base: the velocity terms formed so far at
// the nodes (the learned path's velocity scale is their rms)
static int launch_ns(bs_plan_t P, double *out, const double *base) {
    if (P->prm.ns_mode == BS_NS_ADAPTIVE) {
        launch_ns_adaptive(P, out);
        return BS_OK;
    }
    if (P->prm.ns_mode == BS_NS_MAPPED) {
        launch_ns_mapped(P, out);
        return BS_OK;
    }
    if (!P->mlp) return set_error(P, BS_ESTATE, "BS_NS_MLP plan without bs_set_mlp");
    launch_ns_mlp(P, out, base);
    return BS_OK;
}

// out = base + long-range term (base NULL: out += long-range term); with
// join set, the interpolation waits for that event first
static int long_range(bs_plan_t P, int psi, const double *base, double *out,
                      hipEvent_t join = nullptr) {
    int rc;
    stage_begin(P, 3);
    launch_spread(P);
    stage_end(P, 3);
    if (P->pruned) {
        stage_begin(P, 4);
        pruned_forward(P);
        stage_end(P, 4);
        stage_begin(P, 5);
        pruned_spectral_op(P, psi);
        stage_end(P, 5);
        stage_begin(P, 6);
        pruned_inverse(P);
        stage_end(P, 6);
    } else {
        stage_begin(P, 4);
        if ((rc = fft_forward(P))) return rc;
        stage_end(P, 4);
        stage_begin(P, 5);
        launch_spectral(P, psi);
        stage_end(P, 5);
        stage_begin(P, 6);
        if ((rc = fft_inverse(P))) return rc;
        stage_end(P, 6);
    }
    if (join && (rc = check_hip(P, hipStreamWaitEvent(P->stream, join, 0), "hipStreamWaitEvent")))
        return rc;
    stage_begin(P, 7);
    launch_interp(P, base, out);
    stage_end(P, 7);
    return launch_status(P, "long-range kernels");
}

int bs_velocity(bs_plan_t P, double *v_out) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!P->have_filaments) return set_error(P, BS_ESTATE, "bs_set_filaments not called");
    if (!v_out) return set_error(P, BS_EINVAL, "null output");
    if (P->prm.ns_mode == BS_NS_MLP && !P->mlp)
        return set_error(P, BS_ESTATE, "BS_NS_MLP plan without bs_set_mlp");
    // local - self was formed by set_filaments (d_vls).  The short-range sum
    // and the near-singular correction run on the side stream into
    // tmp3 = (local - self) + short (+ near-singular), concurrently with the
    // spread and the transforms on the plan stream.  Without the correction
    // the interpolation waits for them and writes v = tmp3 + long-range;
    // with it (the side stream's longer chain) the interpolation writes the
    // long-range term alone and tmp3 is added once the side work is in, so
    // that the correction's integrals can run beside the interpolation (the
    // same sum, bitwise).  With per-stage timing on, everything stays on the
    // plan stream, so that each stage's events bracket its own kernels only.
    double *t3 = (double *)P->tmp3.p;
    const bool side = !P->prof;
    int rc;
    if (!side && (rc = join_side(P))) return rc;
    if (side &&
        ((rc = check_hip(P, hipEventRecord(P->ev_fork, P->stream), "hipEventRecord")) ||
         (rc = check_hip(P, hipStreamWaitEvent(P->side, P->ev_fork, 0), "hipStreamWaitEvent"))))
        return rc;
    const hipStream_t plan_stream = P->stream;
    if (side) P->stream = P->side;   // launches below go to the side stream
    rc = BS_OK;
    stage_begin(P, 8);
    launch_pairs(P, 0, (const double *)P->d_vls.p, t3, false);
    stage_end(P, 8);
    if (P->prm.ns_mode != BS_NS_OFF) {
        stage_begin(P, 9);
        rc = launch_ns(P, t3, t3);   // t3 = local - self + short so far
        stage_end(P, 9);
    }
    P->stream = plan_stream;
    const hipError_t ej = side ? hipEventRecord(P->ev_join, P->side) : hipSuccess;
    if (rc || (rc = check_hip(P, ej, "hipEventRecord"))) return rc;
    if (side && P->prm.ns_mode != BS_NS_OFF) {
        fill_f64(P, v_out, 3 * (size_t)P->N, 0.0);
        if ((rc = long_range(P, 0, nullptr, v_out))) return rc;
        if ((rc = check_hip(P, hipStreamWaitEvent(P->stream, P->ev_join, 0), "hipStreamWaitEvent")))
            return rc;
        add_f64(P, v_out, t3, 3 * (size_t)P->N);
    } else if ((rc = long_range(P, 0, t3, v_out, side ? P->ev_join : nullptr))) {
        return rc;
    }
    P->side_pending = false;   // the plan stream now waits for all side work
    if ((rc = launch_status(P, "pair kernel"))) return rc;
    stage_collect(P);
    return BS_OK;
}

int bs_velocity_terms(bs_plan_t P, double *v_local, double *v_short, double *v_long,
                      double *v_self, double *v_ns) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!P->have_filaments) return set_error(P, BS_ESTATE, "bs_set_filaments not called");
    int rc;
    if ((rc = join_side(P))) return rc;
    const size_t n3 = 3 * (size_t)P->N;
    if (v_local) launch_local_self(P, LS_VLOCAL | LS_ASSIGN, 1.0, v_local);
    if (v_self) launch_local_self(P, LS_VSELF | LS_ASSIGN, 1.0, v_self);
    if (v_long) {
        fill_f64(P, v_long, n3, 0.0);
        if ((rc = long_range(P, 0, nullptr, v_long))) return rc;
    }
    if (v_short) {
        fill_f64(P, v_short, n3, 0.0);
        launch_pairs(P, 0, nullptr, v_short, true);
    }
    if (v_ns) {
        fill_f64(P, v_ns, n3, 0.0);
        if (P->prm.ns_mode != BS_NS_OFF &&
            (rc = launch_ns(P, v_ns, (const double *)P->d_vls.p)))
            return rc;
    }
    return launch_status(P, "velocity terms");
}

int bs_energy(bs_plan_t P, double *E_out, double *psi_out) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!P->have_filaments) return set_error(P, BS_ESTATE, "bs_set_filaments not called");
    int rc0 = join_side(P);
    if (rc0) return rc0;
    double *psi = psi_out ? psi_out : (double *)P->tmp3.p;
    launch_local_self(P, LS_VLOCAL | LS_VSELF | LS_PSI | LS_ASSIGN, 1.0, psi);
    int rc = long_range(P, 1, nullptr, psi);
    if (rc) return rc;
    launch_pairs(P, 1, nullptr, psi, true);
    const int nb = 512;
    double *partial = (double *)P->red_tmp.p;   // nb + 1 doubles
    launch_energy(P, psi, partial, nb);
    if ((rc = launch_status(P, "energy kernels"))) return rc;
    if (E_out) {
        if ((rc = check_hip(P, hipMemcpyAsync(E_out, partial + nb, sizeof(double),
                                              hipMemcpyDeviceToHost, P->stream), "copy E")))
            return rc;
    }
    return check_hip(P, hipStreamSynchronize(P->stream), "sync");
}

int bs_vorticity_modes(bs_plan_t P, double *out) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!P->have_filaments) return set_error(P, BS_ESTATE, "bs_set_filaments not called");
    if (!out) return set_error(P, BS_EINVAL, "null output");
    launch_spread(P);
    int rc = fft_forward(P);
    if (rc) return rc;
    launch_modes(P, out);
    return launch_status(P, "mode extraction");
}

int bs_geometry(bs_plan_t P, double *qpos, double *qcharge, double *sdot, double *sddot,
                double *ell) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!P->have_filaments) return set_error(P, BS_ESTATE, "bs_set_filaments not called");
    const size_t N = P->N, Nq = P->Nq;
    struct { void *dst; const void *src; size_t bytes; } cp[5] = {
        {qpos, P->d_qpos.p, 3 * Nq * 8}, {qcharge, P->d_qchg.p, 3 * Nq * 8},
        {sdot, P->d_D.p, 3 * N * 8}, {sddot, P->d_sdd.p, 3 * N * 8}, {ell, P->d_ell.p, N * 8}};
    for (auto &c : cp) {
        if (!c.dst) continue;
        int rc = check_hip(P, hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice,
                                             P->stream), "copy geometry");
        if (rc) return rc;
    }
    return BS_OK;
}

int bs_status(bs_plan_t P) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    int st = 0, rc;
    if ((rc = join_side(P))) return rc;
    if ((rc = check_hip(P, hipMemcpyAsync(&st, P->d_status.p, sizeof(int), hipMemcpyDeviceToHost,
                                          P->stream), "read status")) ||
        (rc = check_hip(P, hipStreamSynchronize(P->stream), "sync")))
        return rc;
    if (st) {
        (void)hipMemsetAsync(P->d_status.p, 0, sizeof(int), P->stream);
        (void)hipStreamSynchronize(P->stream);
        return set_error(P, BS_EINVAL, (st & 1) ? "non-finite node position or zero-length segment"
                                                : "more than 64 near-singular segments at a node");
    }
    return BS_OK;
}

// classical RK4 stage helpers on [N][3] float64 arrays
__global__ void k_axpy_stage(size_t n, const double *__restrict__ x, const double *__restrict__ k,
                             double c, double *__restrict__ y) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + c * k[i];
}
__global__ void k_rk4_final(size_t n, double *__restrict__ x, const double *__restrict__ k1,
                            const double *__restrict__ k2, const double *__restrict__ k3,
                            const double *__restrict__ k4, double dt) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

int bs_rk4_step(bs_plan_t P, int64_t nfil, const int64_t *offsets, double *xyz,
                const double *gamma, double dt) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (!offsets || nfil < 1 || !xyz || !gamma || !std::isfinite(dt))
        return set_error(P, BS_EINVAL, "bad arguments");
    const int64_t N = offsets[nfil];
    const size_t n3 = 3 * (size_t)N;
    int rc;
    if ((rc = ensure<double>(P, P->rk_k, 4 * n3)) || (rc = ensure<double>(P, P->rk_s, n3))) return rc;
    double *k = (double *)P->rk_k.p, *s = (double *)P->rk_s.p;
    const dim3 g((unsigned)((n3 + 255) / 256)), b(256);
    const double c[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    for (int st = 0; st < 4; st++) {
        const double *pos = xyz;
        if (st > 0) {
            hipLaunchKernelGGL(k_axpy_stage, g, b, 0, P->stream, n3, xyz, k + (st - 1) * n3, c[st], s);
            pos = s;
        }
        if ((rc = bs_set_filaments(P, nfil, offsets, pos, gamma))) return rc;
        if ((rc = bs_velocity(P, k + st * n3))) return rc;
    }
    hipLaunchKernelGGL(k_rk4_final, g, b, 0, P->stream, n3, xyz, k, k + n3, k + 2 * n3, k + 3 * n3, dt);
    return launch_status(P, "rk4 kernels");
}

// ---------------------------------------------------------- graph replay
static void drop_graph(bs_plan_t P) {
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
}

int bs_set_graph(bs_plan_t P, int enable) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    if (enable && P->stream == nullptr)
        return set_error(P, BS_EINVAL, "graph replay needs a non-null plan stream");
    if (!enable) drop_graph(P);
    P->use_graph = enable != 0;
    return BS_OK;
}

int bs_step(bs_plan_t P, int64_t nfil, const int64_t *offsets, const double *xyz,
            const double *gamma, double *v_out) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    const bool same = P->gexec && P->have_filaments && P->g_xyz == xyz && P->g_gamma == gamma &&
                      P->g_v == v_out && P->nfil == nfil && offsets &&
                      std::equal(offsets, offsets + nfil + 1, P->off_host.begin());
    if (P->use_graph && !P->prof && same)
        return check_hip(P, hipGraphLaunch(P->gexec, P->stream), "hipGraphLaunch");
    // eager step (also sizes every buffer and uploads the filament structure)
    int rc = bs_set_filaments(P, nfil, offsets, xyz, gamma);
    if (!rc) rc = bs_velocity(P, v_out);
    if (rc || !P->use_graph || P->prof) return rc;
    // capture the same sequence; with unchanged offsets it has no host work
    drop_graph(P);
    hipError_t e = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { P->use_graph = false; return BS_OK; }
    int rc1 = bs_set_filaments(P, nfil, offsets, xyz, gamma);
    int rc2 = rc1 ? rc1 : bs_velocity(P, v_out);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(P->stream, &g);
    if (rc2 || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        P->use_graph = false;        // fall back to eager steps
        return BS_OK;
    }
    if (hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        P->gexec = nullptr;
        P->use_graph = false;
        return BS_OK;
    }
    P->graph = g;
    P->g_xyz = xyz; P->g_gamma = gamma; P->g_v = v_out;
    return BS_OK;
}

int bs_graph_active(bs_plan_t P) { return P && P->gexec ? 1 : 0; }

int bs_set_mlp(bs_plan_t P, bs_mlp_t mlp, const float *err_table, int nbins) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    int want = 0;
    bs_ns_error_bins(nullptr, nullptr, &want);
    if (P->prm.ns_mode != BS_NS_MLP) return set_error(P, BS_ESTATE, "plan is not BS_NS_MLP");
    if (!mlp || !err_table || nbins != want)
        return set_error(P, BS_EINVAL, "need a network and an error table of bs_ns_error_bins bins");
    for (int b = 0; b < nbins; b++)
        if (!(err_table[b] >= 0.0f)) return set_error(P, BS_EINVAL, "error table entry < 0 or NaN");
    // a recorded bs_step graph holds the previous network's buffers and the
    // previous table in its kernel arguments
    drop_graph(P);
    P->mlp = mlp;
    for (int b = 0; b < nbins; b++) P->ns_err[b] = err_table[b];
    return BS_OK;
}

int bs_ns_counts(bs_plan_t P, int64_t *npairs, int64_t *nfallback) {
    if (!P) return set_error(nullptr, BS_EINVAL, "null plan");
    int np = 0, nf = 0, rc;
    if ((rc = join_side(P))) return rc;
    if (P->prm.ns_mode != BS_NS_OFF && P->have_filaments) {
        if ((rc = check_hip(P, hipMemcpyAsync(&np, (int *)P->ns_start.p + P->N, sizeof(int),
                                              hipMemcpyDeviceToHost, P->stream), "read count")))
            return rc;
        int c4[4] = {0, 0, 0, 0};
        if (P->prm.ns_mode == BS_NS_MLP && P->ns_fallback.p &&
            (rc = check_hip(P, hipMemcpyAsync(c4, P->ns_fallback.p, sizeof(c4),
                                              hipMemcpyDeviceToHost, P->stream), "read count")))
            return rc;
        if ((rc = check_hip(P, hipStreamSynchronize(P->stream), "sync"))) return rc;
        // the gate closed: every pair went to the plain integrator
        if (P->prm.ns_mode == BS_NS_MLP) nf = c4[2] ? c4[1] : (c4[3] ? np : 0);
    }
    if (npairs) *npairs = np;
    if (nfallback) *nfallback = nf;
    return BS_OK;
}

int bs_get_params(bs_plan_t P, bs_params *resolved) {
    if (!P || !resolved) return set_error(P, BS_EINVAL, "null argument");
    *resolved = P->prm;
    return BS_OK;
}

int bs_destroy(bs_plan_t P) {
    if (!P) return BS_OK;
    (void)hipStreamSynchronize(P->stream);
    if (P->side) {
        (void)hipStreamSynchronize(P->side);
        (void)hipStreamDestroy(P->side);
    }
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    if (P->ev_ns) (void)hipEventDestroy(P->ev_ns);
    drop_graph(P);
    for (int s = 0; s < BS_NSTAGES; s++) {
        if (P->ev_beg[s]) (void)hipEventDestroy(P->ev_beg[s]);
        if (P->ev_end[s]) (void)hipEventDestroy(P->ev_end[s]);
    }
    if (P->fft_fwd) hipfftDestroy(P->fft_fwd);
    if (P->fft_inv) hipfftDestroy(P->fft_inv);
    DBuf *all[] = {&P->grid, &P->spec, &P->deconv, &P->fftwork, &P->fft_tw, &P->fft_A, &P->fft_B, &P->d_off, &P->d_fil,
                   &P->d_gamma, &P->d_x, &P->d_xn, &P->d_shift, &P->d_dtau, &P->d_D, &P->d_sdd, &P->d_ell,
                   &P->d_qpos, &P->d_qchg, &P->d_status, &P->sp_key, &P->sp_cnt, &P->sp_start,
                   &P->sp_fill, &P->sp_perm, &P->sp_base, &P->sp_ker, &P->sp_q, &P->pq_key,
                   &P->pq_cnt, &P->pq_start, &P->pq_fill, &P->pq_perm, &P->pq_pos, &P->pq_chg,
                   &P->nd_key, &P->nd_cnt, &P->nd_start, &P->nd_fill, &P->nd_perm,
                   &P->scan_tmp, &P->red_tmp, &P->spline_tmp, &P->tmp3, &P->e_D, &P->e_S, &P->d_vls, &P->ns_red, &P->ns_nc, &P->ns_ckey,
                   &P->ns_ccnt, &P->ns_cstart, &P->ns_cfill, &P->ns_cperm, &P->ns_tkey, &P->ns_tcnt,
                   &P->ns_tstart, &P->ns_tfill, &P->ns_tperm, &P->ns_segA, &P->ns_segB, &P->ns_segM, &P->ns_segH, &P->ns_slots,
                   &P->ns_cnt, &P->ns_start, &P->ns_pairs, &P->ns_pnode, &P->ns_pout,
                   &P->ns_X, &P->ns_Y, &P->ns_fallback, &P->ns_learn, &P->ns_fblist, &P->ns_vs, &P->rk_k,
                   &P->rk_s};
    for (DBuf *b : all) release(*b);
    delete P;
    return BS_OK;
}

}  // extern "C"
