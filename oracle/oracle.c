/*
 * Plain FP64 CPU oracle for the Ewald-split Biot-Savart velocity and
 * streamfunction on closed vortex filaments in a triply periodic box.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: it has its own spline (moments form), its own quadrature
 * tables, direct Fourier sums instead of a NUFFT, and a brute-force image loop
 * instead of cell lists.
 *
 * Paper: J. I. Polanco, "Fast and accurate evaluation of Biot-Savart integrals
 * over spatial curves in periodic domains" (arXiv 2406.07366).
 *
 * What each routine follows:
 *   geometry     chord-length parametrisation and periodic cubic spline
 *                (App. B) in moments form, or the periodic quintic spline
 *                of App. B in its B-spline form (Cox-de Boor recursion, dense
 *                interpolation system), Gauss-Legendre rule on each segment
 *                (Sec. 2.7, eq:line_integral_quadrature); vector charges
 *                q = Gamma w_i dtau_j s'_ij (Sec. 3.3, eq:vorticity_fourier_coefs).
 *   local        eq:BS_local and eq:streamfunction_local (Sec. 2.4, 2.6).
 *   short-range  eq:velocity_shortrange, eq:streamfunction_shortrange with
 *                g_sr, f_sr = erfc (eq:ewald_derivative_weight_functions),
 *                summed over every periodic image within r_c, local segments
 *                excluded for the unshifted image only.
 *   long-range   Fourier coefficients by direct sums over the quadrature
 *                points (eq:vorticity_fourier_coefs), Gaussian filter and
 *                curl/Poisson in Fourier space
 *                (eq:velocity_longrange_physical), cubic mode truncation
 *                |m_i| <= K in every axis, k = 0 removed.
 *   self         eq:velocity_longrange_self, eq:streamfunction_longrange_self
 *                on the same 2Q quadrature points the long-range part uses.
 *   brute        the unsplit sum (alpha = 0) over cubic shells of images.
 *   energy       eq:kinetic_energy_streamfunction: psi interpolated between
 *                the nodes by the curve's own spline, Q-point rule per segment.
 *   impulse      p = (1/2V) sum Gamma s x ds (Sec. 5.2).
 *   near-singular  exact integral of the full kernel over one spline segment
 *                (adaptive Gauss-Kronrod 7/15) minus its Q-point sum; and
 *                the closed-form Biot-Savart integral of a straight segment.
 *                The paper does not define this correction; the definition used is
 *                stated above or_ns_correction.
 *
 * Conventions: node arrays are [N][3] row-major, filaments are CSR
 * (off[nfil+1]); segment j joins node j to the next node of its filament;
 * quadrature point q = j*Q + i lies on segment j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>
#include <omp.h>

#define OR_PI 3.14159265358979323846264338327950288

typedef struct {
    int64_t nfil, N, Nq;
    int Q, order;      /* order 4: cubic (moments form); 6: quintic (B-splines) */
    double L, a, delta;
    int64_t *off;      /* nfil+1 */
    int64_t *fil;      /* N: filament of node */
    double *gamma;     /* nfil */
    double *x;         /* N*3 node positions */
    double *tau;       /* N: parameter at node */
    double *dtau;      /* N: tau_{j+1}-tau_j */
    double *M;         /* N*3 second derivatives at nodes (moments) */
    double *C;         /* N*3 B-spline coefficients (order 6 only) */
    double *shift;     /* nfil*3: s(tau + T) = s(tau) + shift (n L; 0: closed) */
    double *T;         /* nfil: period of the parameter */
    double *sd;        /* N*3 first derivative at nodes */
    double *ell;       /* N: segment length by the Q-point rule */
    double *qx;        /* Nq*3 quadrature point positions */
    double *qs;        /* Nq*3 derivative at quadrature points */
    double *qc;        /* Nq*3 vector charges Gamma*w*dtau*s' */
    double gl_h[8], gl_w[8];
} or_t;

/* ---------------------------------------------------------------- small vec */
static inline void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline double norm3(const double *a) { return sqrt(dot3(a, a)); }

static inline int64_t next_node(const or_t *o, int64_t j) {
    int64_t f = o->fil[j];
    return (j + 1 < o->off[f + 1]) ? j + 1 : o->off[f];
}
static inline int64_t prev_node(const or_t *o, int64_t j) {
    int64_t f = o->fil[j];
    return (j > o->off[f]) ? j - 1 : o->off[f + 1] - 1;
}

/* Sec. 2.1: a filament satisfies s(tau + T) = s(tau) + n L (n = 0: closed).
 * The node after the last one is the first node moved by n L; wrap(o, j)
 * is 1 when segment j is that closing segment. */
static inline int wraps(const or_t *o, int64_t j) {
    return j + 1 == o->off[o->fil[j] + 1];
}

/* position of the end of segment j in the frame of its start (nodal data
 * other than positions repeats with period T: shifted = 0) */
static inline void seg_end(const or_t *o, const double *data, int64_t j, int shifted,
                           double *out) {
    int64_t jn = next_node(o, j);
    const double *sh = o->shift + 3 * o->fil[j];
    int w = shifted && wraps(o, j);
    for (int c = 0; c < 3; c++) out[c] = data[3 * jn + c] + (w ? sh[c] : 0.0);
}

/* offset that brings the points of segment seg (adjacent to node i) into
 * the frame of node i: -n L for the closing segment ending at the first
 * node, else 0 */
static inline void adj_offset(const or_t *o, int64_t i, int64_t seg, double *E) {
    int64_t f = o->fil[i];
    int w = (i == o->off[f]) && seg == prev_node(o, i);
    for (int c = 0; c < 3; c++) E[c] = w ? -o->shift[3 * f + c] : 0.0;
}

/* ------------------------------------------------- Gauss-Legendre on [0,1] */
/* Closed forms of the Legendre roots and weights, mapped from [-1,1]. */
int or_gl_rule(int Q, double *h, double *w) {
    double x[4], ww[4];
    switch (Q) {
    case 1: x[0] = 0; ww[0] = 2; break;
    case 2: x[0] = -1 / sqrt(3.0); x[1] = -x[0]; ww[0] = ww[1] = 1; break;
    case 3:
        x[0] = -sqrt(3.0 / 5.0); x[1] = 0; x[2] = -x[0];
        ww[0] = ww[2] = 5.0 / 9.0; ww[1] = 8.0 / 9.0; break;
    case 4: {
        double p = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(6.0 / 5.0));
        double q = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(6.0 / 5.0));
        x[0] = -q; x[1] = -p; x[2] = p; x[3] = q;
        ww[0] = ww[3] = (18.0 - sqrt(30.0)) / 36.0;
        ww[1] = ww[2] = (18.0 + sqrt(30.0)) / 36.0; break;
    }
    default: return -1;
    }
    for (int i = 0; i < Q; i++) { h[i] = 0.5 * (x[i] + 1.0); w[i] = 0.5 * ww[i]; }
    return 0;
}

/* ------------------------------------------- cyclic tridiagonal (App. B)  */
/* Solves a_i x_{i-1} + b_i x_i + c_i x_{i+1} = r_i, indices mod n (n >= 3),
 * by the Sherman-Morrison correction of a plain tridiagonal Thomas solve.
 * a, b, c are read only; r is overwritten with the solution.  work >= 3n. */
static void cyclic_tridiag(int64_t n, const double *a, const double *b,
                           const double *c, double *r, double *work) {
    double *bb = work, *y = work + n, *z = work + 2 * n;
    double gam = -b[0];
    double top = a[0];          /* row 0, column n-1 */
    double bot = c[n - 1];      /* row n-1, column 0 */
    for (int64_t i = 0; i < n; i++) bb[i] = b[i];
    bb[0] -= gam;
    bb[n - 1] -= top * bot / gam;
    /* Thomas on (a, bb, c) for two right-hand sides: r and u */
    for (int64_t i = 0; i < n; i++) { y[i] = r[i]; z[i] = 0.0; }
    z[0] = gam; z[n - 1] = bot;
    /* forward sweep, storing modified c in work via cp (reuse r? keep local) */
    double *cp = (double *)malloc(sizeof(double) * n);
    double den = bb[0];
    cp[0] = c[0] / den; y[0] /= den; z[0] /= den;
    for (int64_t i = 1; i < n; i++) {
        den = bb[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / den : 0.0;
        y[i] = (y[i] - a[i] * y[i - 1]) / den;
        z[i] = (z[i] - a[i] * z[i - 1]) / den;
    }
    for (int64_t i = n - 2; i >= 0; i--) {
        y[i] -= cp[i] * y[i + 1];
        z[i] -= cp[i] * z[i + 1];
    }
    free(cp);
    /* v = [1, 0, ..., 0, top/gam] */
    double vy = y[0] + top / gam * y[n - 1];
    double vz = z[0] + top / gam * z[n - 1];
    double f = vy / (1.0 + vz);
    for (int64_t i = 0; i < n; i++) r[i] = y[i] - f * z[i];
}

/* exported for a direct test against a dense solve */
void or_cyclic_tridiag(int64_t n, const double *a, const double *b,
                       const double *c, double *r) {
    double *w = (double *)malloc(sizeof(double) * 3 * n);
    cyclic_tridiag(n, a, b, c, r, w);
    free(w);
}

/* ------------------------------------------ spline on one segment (moments) */
/* Periodic interpolating cubic spline in second-derivative ("moments") form:
 * on [tau_j, tau_j + h], t = tau - tau_j,
 *   s(t) = M_j (h-t)^3/(6h) + M_{j+1} t^3/(6h)
 *        + (s_j/h - M_j h/6)(h-t) + (s_{j+1}/h - M_{j+1} h/6) t.
 * deriv = 0, 1, 2 returns s, ds/dtau, d2s/dtau2. */
/* ------------------------------------------- quintic B-splines (App. B) */
/* B-spline of order k on the k+1 knots kn[0..k], or its d-th derivative, at
 * x: Cox-de Boor recursion, half-open intervals [kn_i, kn_{i+1}). */
static double bspl(const double *kn, int k, double x, int d) {
    if (d == 0) {
        if (k == 1) return (kn[0] <= x && x < kn[1]) ? 1.0 : 0.0;
        double v = 0.0;
        if (kn[k - 1] > kn[0]) v += (x - kn[0]) / (kn[k - 1] - kn[0]) * bspl(kn, k - 1, x, 0);
        if (kn[k] > kn[1]) v += (kn[k] - x) / (kn[k] - kn[1]) * bspl(kn + 1, k - 1, x, 0);
        return v;
    }
    double v = 0.0;
    if (kn[k - 1] > kn[0]) v += bspl(kn, k - 1, x, d - 1) / (kn[k - 1] - kn[0]);
    if (kn[k] > kn[1]) v -= bspl(kn + 1, k - 1, x, d - 1) / (kn[k] - kn[1]);
    return (k - 1) * v;
}

/* knot p of filament f, periodically extended: t_{p+n} = t_p + T */
static double knot(const or_t *o, int64_t f, int64_t p) {
    int64_t b = o->off[f], n = o->off[f + 1] - b;
    int64_t q = p % n;
    if (q < 0) q += n;
    return o->tau[b + q] + (double)((p - q) / n) * o->T[f];
}

/* knots of basis function jp (unwrapped index) of order k: t_{jp-k/2..jp+k/2} */
static void basis_knots(const or_t *o, int64_t f, int64_t jp, int k, double *kn) {
    for (int i = 0; i <= k; i++) kn[i] = knot(o, f, jp - k / 2 + i);
}

/* s = sum_j c_j b_j(tau) (eq:spline_from_bspline_basis) at tau = tau_j + t:
 * the basis functions whose support covers [t_j, t_{j+1}) are j-2..j+3 */
static void bspline_eval(const or_t *o, const double *coef, int64_t j, double t, int deriv,
                         int shifted, double *out) {
    int64_t f = o->fil[j], b = o->off[f], n = o->off[f + 1] - b, jl = j - b;
    double x = o->tau[j] + t, kn[8];
    out[0] = out[1] = out[2] = 0.0;
    for (int64_t jp = jl - 2; jp <= jl + 3; jp++) {
        basis_knots(o, f, jp, 6, kn);
        double w = bspl(kn, 6, x, deriv);
        int64_t q = ((jp % n) + n) % n, k = (jp - q) / n;
        /* c_{jp} = c_{jp mod n} + k n L for positions (Sec. 2.1) */
        for (int c = 0; c < 3; c++)
            out[c] += w * (coef[3 * (b + q) + c] + (shifted ? k * o->shift[3 * f + c] : 0.0));
    }
}

/* dense Gaussian elimination with partial pivoting, nrhs right-hand sides
 * stored column-wise in r[n][nrhs]; A (n x n, row-major) is destroyed */
static int dense_solve(int64_t n, double *A, double *r, int nrhs) {
    for (int64_t c = 0; c < n; c++) {
        int64_t p = c;
        for (int64_t i = c + 1; i < n; i++)
            if (fabs(A[i * n + c]) > fabs(A[p * n + c])) p = i;
        if (A[p * n + c] == 0.0) return -1;
        if (p != c) {
            for (int64_t k = 0; k < n; k++) {
                double t = A[c * n + k]; A[c * n + k] = A[p * n + k]; A[p * n + k] = t;
            }
            for (int k = 0; k < nrhs; k++) {
                double t = r[c * nrhs + k]; r[c * nrhs + k] = r[p * nrhs + k]; r[p * nrhs + k] = t;
            }
        }
        for (int64_t i = c + 1; i < n; i++) {
            double m = A[i * n + c] / A[c * n + c];
            if (m == 0.0) continue;
            for (int64_t k = c; k < n; k++) A[i * n + k] -= m * A[c * n + k];
            for (int k = 0; k < nrhs; k++) r[i * nrhs + k] -= m * r[c * nrhs + k];
        }
    }
    for (int64_t c = n - 1; c >= 0; c--) {
        for (int k = 0; k < nrhs; k++) {
            double v = r[c * nrhs + k];
            for (int64_t i = c + 1; i < n; i++) v -= A[c * n + i] * r[i * nrhs + k];
            r[c * nrhs + k] = v / A[c * n + c];
        }
    }
    return 0;
}

/* interpolation A c = d with A_ij = b_j(tau_i) (App. B) for the nodal data d
 * (3 components) of filament f; coefficients into coef */
static int quintic_fit(const or_t *o, int64_t f, const double *data, int shifted,
                       double *coef) {
    int64_t b = o->off[f], n = o->off[f + 1] - b;
    double *A = (double *)calloc((size_t)(n * n), sizeof(double));
    double *r = (double *)malloc(sizeof(double) * 3 * n), kn[8];
    for (int64_t i = 0; i < n; i++) {
        for (int c = 0; c < 3; c++) r[3 * i + c] = data[3 * (b + i) + c];
        for (int64_t jp = i - 3; jp <= i + 3; jp++) {
            basis_knots(o, f, jp, 6, kn);
            int64_t q = ((jp % n) + n) % n, k = (jp - q) / n;
            double w = bspl(kn, 6, o->tau[b + i], 0);
            A[i * n + q] += w;
            /* the wrapped coefficients carry k n L: moved to the right side */
            if (shifted && k != 0)
                for (int c = 0; c < 3; c++) r[3 * i + c] -= w * k * o->shift[3 * f + c];
        }
    }
    int rc = dense_solve(n, A, r, 3);
    memcpy(coef + 3 * b, r, sizeof(double) * 3 * n);
    free(A); free(r);
    return rc;
}

/* periodic cubic spline through the nodal data d of filament f in moments
 * form: h_{k-1} M_{k-1} + 2(h_{k-1}+h_k) M_k + h_k M_{k+1}
 *     = 6[(d_{k+1}-d_k)/h_k - (d_k-d_{k-1})/h_{k-1}]  (M = d'' at the nodes) */
static void cubic_fit(const or_t *o, int64_t f, const double *data, int shifted, double *M) {
    int64_t b = o->off[f], n = o->off[f + 1] - b;
    double *aa = (double *)malloc(sizeof(double) * n);
    double *bb = (double *)malloc(sizeof(double) * n);
    double *cc = (double *)malloc(sizeof(double) * n);
    double *rr = (double *)malloc(sizeof(double) * n);
    double *wk = (double *)malloc(sizeof(double) * 3 * n);
    for (int64_t k = 0; k < n; k++) {
        double hm = o->dtau[b + (k + n - 1) % n], hk = o->dtau[b + k];
        aa[k] = hm; bb[k] = 2.0 * (hm + hk); cc[k] = hk;
    }
    for (int c = 0; c < 3; c++) {
        for (int64_t k = 0; k < n; k++) {
            int64_t j = b + k, jp = b + (k + n - 1) % n;
            double hm = o->dtau[jp], hk = o->dtau[j], en[3], ep[3];
            seg_end(o, data, j, shifted, en);     /* s_{k+1} in the frame of s_k */
            seg_end(o, data, jp, shifted, ep);    /* s_k in the frame of s_{k-1} */
            rr[k] = 6.0 * ((en[c] - data[3 * j + c]) / hk - (ep[c] - data[3 * jp + c]) / hm);
        }
        cyclic_tridiag(n, aa, bb, cc, rr, wk);
        for (int64_t k = 0; k < n; k++) M[3 * (b + k) + c] = rr[k];
    }
    free(aa); free(bb); free(cc); free(rr); free(wk);
}

/* the spline through nodal data (aux = its moments for order 4, its B-spline
 * coefficients for order 6) on segment j at tau = tau_j + t */
static void spline_eval_data(const or_t *o, const double *data, const double *aux, int64_t j,
                             double t, int deriv, int shifted, double *out) {
    if (o->order == 6) {
        bspline_eval(o, aux, j, t, deriv, shifted, out);
        return;
    }
    int64_t jn = next_node(o, j);
    double h = o->dtau[j], sn[3];
    const double *Mj = aux + 3 * j, *Mn = aux + 3 * jn;
    const double *sj = data + 3 * j;
    seg_end(o, data, j, shifted, sn);
    double u = h - t;
    for (int c = 0; c < 3; c++) {
        double A = sj[c] / h - Mj[c] * h / 6.0;
        double B = sn[c] / h - Mn[c] * h / 6.0;
        if (deriv == 0)
            out[c] = Mj[c] * u * u * u / (6 * h) + Mn[c] * t * t * t / (6 * h) + A * u + B * t;
        else if (deriv == 1)
            out[c] = -Mj[c] * u * u / (2 * h) + Mn[c] * t * t / (2 * h) - A + B;
        else
            out[c] = Mj[c] * u / h + Mn[c] * t / h;
    }
}

/* the curve: s, ds/dtau or d2s/dtau2 on segment j at tau = tau_j + t */
static void seg_eval(const or_t *o, int64_t j, double t, int deriv, double *out) {
    spline_eval_data(o, o->x, o->order == 6 ? o->C : o->M, j, t, deriv, 1, out);
}

void or_spline_eval(const void *h, int64_t seg, double u, int deriv, double *out) {
    const or_t *o = (const or_t *)h;
    seg_eval(o, seg, u * o->dtau[seg], deriv, out);
}

/* --------------------------------------------------------------- geometry */
void or_free(void *h) {
    or_t *o = (or_t *)h;
    if (!o) return;
    free(o->off); free(o->fil); free(o->gamma); free(o->x); free(o->tau);
    free(o->dtau); free(o->M); free(o->sd); free(o->ell); free(o->C); free(o->T);
    free(o->shift);
    free(o->qx); free(o->qs); free(o->qc);
    free(o);
}

void *or_new(int64_t nfil, const int64_t *off, const double *xyz,
             const double *gamma, double L, double a, double delta, int Q, int order,
             const int64_t *periods) {
    if (nfil < 1 || Q < 1 || Q > 4 || (order != 4 && order != 6)) return NULL;
    for (int64_t f = 0; f < nfil; f++)
        if (off[f + 1] - off[f] < (order == 6 ? 6 : 3)) return NULL;
    or_t *o = (or_t *)calloc(1, sizeof(or_t));
    o->nfil = nfil; o->N = off[nfil]; o->Q = Q; o->Nq = o->N * Q; o->order = order;
    o->L = L; o->a = a; o->delta = delta;
    int64_t N = o->N;
    o->off = (int64_t *)malloc(sizeof(int64_t) * (nfil + 1));
    memcpy(o->off, off, sizeof(int64_t) * (nfil + 1));
    o->fil = (int64_t *)malloc(sizeof(int64_t) * N);
    o->gamma = (double *)malloc(sizeof(double) * nfil);
    memcpy(o->gamma, gamma, sizeof(double) * nfil);
    o->x = (double *)malloc(sizeof(double) * 3 * N);
    memcpy(o->x, xyz, sizeof(double) * 3 * N);
    o->tau = (double *)malloc(sizeof(double) * N);
    o->dtau = (double *)malloc(sizeof(double) * N);
    o->M = (double *)malloc(sizeof(double) * 3 * N);
    o->C = (double *)calloc((size_t)(3 * N), sizeof(double));
    o->T = (double *)malloc(sizeof(double) * nfil);
    o->shift = (double *)calloc((size_t)(3 * nfil), sizeof(double));
    if (periods)
        for (int64_t k = 0; k < 3 * nfil; k++) o->shift[k] = (double)periods[k] * L;
    o->sd = (double *)malloc(sizeof(double) * 3 * N);
    o->ell = (double *)malloc(sizeof(double) * N);
    o->qx = (double *)malloc(sizeof(double) * 3 * o->Nq);
    o->qs = (double *)malloc(sizeof(double) * 3 * o->Nq);
    o->qc = (double *)malloc(sizeof(double) * 3 * o->Nq);
    or_gl_rule(Q, o->gl_h, o->gl_w);
    for (int64_t f = 0; f < nfil; f++)
        for (int64_t j = off[f]; j < off[f + 1]; j++) o->fil[j] = f;

    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t f = 0; f < nfil; f++) {
        int64_t b = off[f], n = off[f + 1] - off[f];
        /* chord-length parametrisation (App. B) */
        o->tau[b] = 0.0;
        for (int64_t k = 0; k < n; k++) {
            int64_t j = b + k, jn = b + (k + 1) % n;
            double e[3];
            seg_end(o, o->x, j, 1, e);
            double d[3] = {e[0] - o->x[3 * j], e[1] - o->x[3 * j + 1], e[2] - o->x[3 * j + 2]};
            o->dtau[j] = norm3(d);
            if (!(o->dtau[j] > 0.0)) bad = 1;
            if (k + 1 < n) o->tau[jn] = o->tau[j] + o->dtau[j];
        }
        o->T[f] = o->tau[b + n - 1] + o->dtau[b + n - 1];
        if (bad) continue;
        if (order == 6) {
            if (quintic_fit(o, f, o->x, 1, o->C)) bad = 1;
            for (int64_t k = 0; k < n; k++)
                bspline_eval(o, o->C, b + k, 0.0, 2, 1, o->M + 3 * (b + k));
        } else {
            cubic_fit(o, f, o->x, 1, o->M);
        }
    }
    if (bad) { or_free(o); return NULL; }

#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; j++) {
        double h = o->dtau[j];
        double gam = o->gamma[o->fil[j]];
        seg_eval(o, j, 0.0, 1, o->sd + 3 * j);
        double ell = 0.0;
        for (int i = 0; i < Q; i++) {
            int64_t q = j * Q + i;
            double t = o->gl_h[i] * h;
            seg_eval(o, j, t, 0, o->qx + 3 * q);
            seg_eval(o, j, t, 1, o->qs + 3 * q);
            for (int c = 0; c < 3; c++) o->qc[3 * q + c] = gam * o->gl_w[i] * h * o->qs[3 * q + c];
            ell += o->gl_w[i] * norm3(o->qs + 3 * q) * h;
        }
        o->ell[j] = ell;
    }
    return o;
}

int64_t or_nquad(const void *h) { return ((const or_t *)h)->Nq; }

void or_get_quad(const void *h, double *pos, double *deriv, double *charge) {
    const or_t *o = (const or_t *)h;
    if (pos) memcpy(pos, o->qx, sizeof(double) * 3 * o->Nq);
    if (deriv) memcpy(deriv, o->qs, sizeof(double) * 3 * o->Nq);
    if (charge) memcpy(charge, o->qc, sizeof(double) * 3 * o->Nq);
}

void or_get_nodes(const void *h, double *tau, double *dtau, double *sdot,
                  double *sddot, double *ell) {
    const or_t *o = (const or_t *)h;
    int64_t N = o->N;
    if (tau) memcpy(tau, o->tau, sizeof(double) * N);
    if (dtau) memcpy(dtau, o->dtau, sizeof(double) * N);
    if (sdot) memcpy(sdot, o->sd, sizeof(double) * 3 * N);
    if (sddot) memcpy(sddot, o->M, sizeof(double) * 3 * N);
    if (ell) memcpy(ell, o->ell, sizeof(double) * N);
}

/* ------------------------------------------------------------ local terms */
/* eq:BS_local and eq:streamfunction_local; s' x s'' = sdot x sddot/|sdot|^3. */
void or_local(const void *h, int64_t nt, const int64_t *tgt, double *v, double *psi) {
    const or_t *o = (const or_t *)h;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t];
        double gam = o->gamma[o->fil[i]];
        const double *sd = o->sd + 3 * i, *sdd = o->M + 3 * i;
        double lm = o->ell[prev_node(o, i)], lp = o->ell[i];
        double lg = log(2.0 * sqrt(lm * lp) / o->a);
        double sn = norm3(sd), b[3];
        cross3(sd, sdd, b);
        for (int c = 0; c < 3; c++) {
            if (v) v[3 * t + c] = gam / (4 * OR_PI) * b[c] / (sn * sn * sn) * (lg - o->delta);
            if (psi) psi[3 * t + c] = gam / (2 * OR_PI) * sd[c] / sn * (lg - (o->delta - 1.0));
        }
    }
}

/* Local terms with the local segments subdivided (Sec. 5.2): on each of the
 * two segments next to node i, the fraction eps of its parameter interval
 * that touches node i is the central portion, treated by the Taylor
 * expansion (eq:BS_local, eq:streamfunction_local with l-, l+ the arc lengths
 * of the two central portions); the rest of each segment is integrated with
 * the unsplit kernels (eq:BS, eq:streamfunction_integral) by 3-point
 * Gauss-Legendre rules on panels graded towards the node: in the distance
 * u from the node (in units of the segment's parameter interval) the panels
 * are [eps, 2 eps], [2 eps, 4 eps], ..., the last one ending at u = 1, so
 * that each panel's distance to the node is at least its own length (the
 * integrand behaves like 1/u there).  Arc lengths of the central portions
 * use the 3-point rule.  eps = 1 gives back or_local up to the rule used for
 * l-, l+. */
void or_local_sub(const void *h, double eps, int64_t nt, const int64_t *tgt, double *v,
                  double *psi) {
    const or_t *o = (const or_t *)h;
    double g3h[4], g3w[4];
    or_gl_rule(3, g3h, g3w);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t], jm = prev_node(o, i);
        double gam = o->gamma[o->fil[i]];
        const double *si = o->x + 3 * i, *sd = o->sd + 3 * i, *sdd = o->M + 3 * i;
        double hm = o->dtau[jm], hp = o->dtau[i];
        /* central portions: [hm (1-eps), hm] on segment jm, [0, eps hp] on segment i */
        double lm = 0.0, lp = 0.0, d[3];
        for (int k = 0; k < 3; k++) {
            seg_eval(o, jm, hm * (1.0 - eps) + g3h[k] * eps * hm, 1, d);
            lm += g3w[k] * eps * hm * norm3(d);
            seg_eval(o, i, g3h[k] * eps * hp, 1, d);
            lp += g3w[k] * eps * hp * norm3(d);
        }
        double lg = log(2.0 * sqrt(lm * lp) / o->a);
        double sn = norm3(sd), b[3];
        cross3(sd, sdd, b);
        double vv[3], pp[3];
        for (int c = 0; c < 3; c++) {
            vv[c] = gam / (4 * OR_PI) * b[c] / (sn * sn * sn) * (lg - o->delta);
            pp[c] = gam / (2 * OR_PI) * sd[c] / sn * (lg - (o->delta - 1.0));
        }
        /* remaining portions, distance u from the node in [eps, 1]: on
         * segment i at t = u hp, on segment jm at t = (1 - u) hm */
        for (int side = 0; side < 2; side++) {
            int64_t j = side ? i : jm;
            double hs = side ? hp : hm, E[3];
            adj_offset(o, i, j, E);
            for (double u0 = eps; u0 < 1.0; u0 *= 2.0) {
                double u1 = fmin(2.0 * u0, 1.0);
                for (int k = 0; k < 3; k++) {
                    double u = u0 + g3h[k] * (u1 - u0), x[3], sdq[3], r[3], rx[3];
                    double t = side ? u * hs : (1.0 - u) * hs;
                    seg_eval(o, j, t, 0, x);
                    seg_eval(o, j, t, 1, sdq);
                    for (int c = 0; c < 3; c++) r[c] = x[c] + E[c] - si[c];
                    double rn = norm3(r), wq = gam * g3w[k] * (u1 - u0) * hs / (4 * OR_PI);
                    cross3(r, sdq, rx);
                    for (int c = 0; c < 3; c++) {
                        vv[c] += wq * rx[c] / (rn * rn * rn);
                        pp[c] += wq * sdq[c] / rn;
                    }
                }
            }
        }
        for (int c = 0; c < 3; c++) {
            if (v) v[3 * t + c] = vv[c];
            if (psi) psi[3 * t + c] = pp[c];
        }
    }
}

/* ------------------------------------------------- Ewald weight functions */
/* g_sr = erfc(x) + 2x/sqrt(pi) exp(-x^2), g_lr = erf(x) - 2x/sqrt(pi) exp(-x^2)
 * (eq:ewald_derivative_weight_functions), x = alpha r.  For x < 0.5 g_lr is
 * summed from its Taylor series (2/sqrt(pi)) sum_{n>=1} (-1)^{n+1} 2n
 * x^{2n+1}/(n!(2n+1)) to avoid the cancellation of the two terms. */
double or_g_lr(double x) {
    if (x < 0.5) {
        double term = x, sum = 0.0, x2 = x * x;   /* term = x^{2n+1}/n! */
        for (int n = 1; n < 40; n++) {
            term *= x2 / n;
            double add = ((n & 1) ? 1.0 : -1.0) * 2.0 * n * term / (2.0 * n + 1.0);
            sum += add;
            if (fabs(add) < 1e-18 * fabs(sum)) break;
        }
        return 2.0 / sqrt(OR_PI) * sum;
    }
    return erf(x) - 2.0 * x / sqrt(OR_PI) * exp(-x * x);
}
double or_g_sr(double x) { return erfc(x) + 2.0 * x / sqrt(OR_PI) * exp(-x * x); }

/* ---------------------------------------------------------- short range */
/* eq:velocity_shortrange / eq:streamfunction_shortrange as quadrature sums,
 * over every periodic image with |r| < rc.  alpha = 0 gives the unsplit
 * kernels restricted to the ball of radius rc. */
void or_shortrange(const void *h, double alpha, double rc, int64_t nt,
                   const int64_t *tgt, double *v, double *psi) {
    const or_t *o = (const or_t *)h;
    double L = o->L;
    int nm = (int)ceil(rc / L - 0.5);
    if (nm < 0) nm = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t], ip = prev_node(o, i);
        const double *xi = o->x + 3 * i;
        double av[3] = {0, 0, 0}, ap[3] = {0, 0, 0};
        for (int64_t q = 0; q < o->Nq; q++) {
            int64_t seg = q / o->Q;
            int adj = (seg == i || seg == ip);
            double E[3] = {0, 0, 0};   /* image holding the local copy of an adjacent segment */
            if (adj) adj_offset(o, i, seg, E);
            double d0[3], sh[3];
            for (int c = 0; c < 3; c++) {
                d0[c] = o->qx[3 * q + c] - xi[c];
                sh[c] = -L * nearbyint(d0[c] / L);   /* minimum-image shift */
            }
            for (int nx = -nm; nx <= nm; nx++)
            for (int ny = -nm; ny <= nm; ny++)
            for (int nz = -nm; nz <= nm; nz++) {
                double r[3] = {d0[0] + sh[0] + nx * L, d0[1] + sh[1] + ny * L,
                               d0[2] + sh[2] + nz * L};
                int unshifted = (fabs(sh[0] + nx * L - E[0]) < 0.5 * L &&
                                 fabs(sh[1] + ny * L - E[1]) < 0.5 * L &&
                                 fabs(sh[2] + nz * L - E[2]) < 0.5 * L);
                if (adj && unshifted) continue;
                double r2 = dot3(r, r);
                if (r2 >= rc * rc || r2 == 0.0) continue;
                double rr = sqrt(r2);
                const double *qc = o->qc + 3 * q;
                double gsr = (alpha > 0) ? or_g_sr(alpha * rr) : 1.0;
                double fsr = (alpha > 0) ? erfc(alpha * rr) : 1.0;
                double cr[3];
                cross3(r, qc, cr);
                for (int c = 0; c < 3; c++) {
                    av[c] += gsr * cr[c] / (r2 * rr);
                    ap[c] += fsr * qc[c] / rr;
                }
            }
        }
        for (int c = 0; c < 3; c++) {
            if (v) v[3 * t + c] = av[c] / (4 * OR_PI);
            if (psi) psi[3 * t + c] = ap[c] / (4 * OR_PI);
        }
    }
}

/* ---------------------------------------------------------- self terms */
/* eq:velocity_longrange_self / eq:streamfunction_longrange_self on the 2Q
 * quadrature points of the two segments adjacent to the node. */
void or_selfcorr(const void *h, double alpha, int64_t nt, const int64_t *tgt,
                 double *v, double *psi) {
    const or_t *o = (const or_t *)h;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t], segs[2] = {prev_node(o, i), i};
        const double *xi = o->x + 3 * i;
        double av[3] = {0, 0, 0}, ap[3] = {0, 0, 0};
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < o->Q; k++) {
                int64_t q = segs[s] * o->Q + k;
                double r[3], cr[3], E[3];
                adj_offset(o, i, segs[s], E);
                for (int c = 0; c < 3; c++) r[c] = o->qx[3 * q + c] + E[c] - xi[c];
                double rr = norm3(r);
                const double *qc = o->qc + 3 * q;
                cross3(r, qc, cr);
                double x = alpha * rr;
                /* g_lr(x)/r^3 and erf(x)/r */
                double glr = or_g_lr(x);
                for (int c = 0; c < 3; c++) {
                    av[c] += glr * cr[c] / (rr * rr * rr);
                    ap[c] += erf(x) * qc[c] / rr;
                }
            }
        for (int c = 0; c < 3; c++) {
            if (v) v[3 * t + c] = av[c] / (4 * OR_PI);
            if (psi) psi[3 * t + c] = ap[c] / (4 * OR_PI);
        }
    }
}

/* ---------------------------------------------------------- long range */
/* Half-space mode index: modes (mx,my,mz) with mz>0, or mz==0 & my>0, or
 * mz==my==0 & mx>0; k = 2 pi m / L.  The other half follows by conjugation. */
typedef struct { int mx, my, mz; } mode_t3;

static int64_t half_modes(int K, mode_t3 **out) {
    int64_t cap = (int64_t)(2 * K + 1) * (2 * K + 1) * (K + 1), n = 0;
    mode_t3 *m = (mode_t3 *)malloc(sizeof(mode_t3) * cap);
    for (int mz = 0; mz <= K; mz++)
        for (int my = -K; my <= K; my++)
            for (int mx = -K; mx <= K; mx++) {
                if (mz == 0 && (my < 0 || (my == 0 && mx <= 0))) continue;
                m[n].mx = mx; m[n].my = my; m[n].mz = mz; n++;
            }
    *out = m;
    return n;
}

/* omega_hat_k = (1/V) sum_q q_q exp(-i k.s_q), for the half-space modes. */
static void omega_hat(const or_t *o, int K, int64_t nm, const mode_t3 *modes,
                      double complex *w /* nm*3 */) {
    double L = o->L, k0 = 2 * OR_PI / L, V = L * L * L;
    int nthr = omp_get_max_threads();
    int W = 2 * K + 1;
    double complex *acc = (double complex *)calloc((size_t)nthr * nm * 3, sizeof(double complex));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double complex *my = acc + (size_t)tid * nm * 3;
        double complex *e = (double complex *)malloc(sizeof(double complex) * 3 * W);
#pragma omp for schedule(static)
        for (int64_t q = 0; q < o->Nq; q++) {
            for (int c = 0; c < 3; c++)
                for (int m = -K; m <= K; m++)
                    e[c * W + m + K] = cexp(-I * (k0 * m * o->qx[3 * q + c]));
            const double *qc = o->qc + 3 * q;
            for (int64_t t = 0; t < nm; t++) {
                double complex ph = e[modes[t].mx + K] * e[W + modes[t].my + K] *
                                    e[2 * W + modes[t].mz + K];
                my[3 * t + 0] += qc[0] * ph;
                my[3 * t + 1] += qc[1] * ph;
                my[3 * t + 2] += qc[2] * ph;
            }
        }
        free(e);
    }
    for (int64_t t = 0; t < 3 * nm; t++) {
        double complex s = 0;
        for (int th = 0; th < nthr; th++) s += acc[(size_t)th * nm * 3 + t];
        w[t] = s / V;
    }
    free(acc);
}

/* v_lr and psi_lr at target nodes: v_hat = i k x w_hat exp(-k^2/4a^2)/k^2,
 * psi_hat = w_hat exp(-k^2/4a^2)/k^2; f(x) = 2 Re sum_half f_hat e^{ik.x}. */
void or_longrange(const void *h, double alpha, int K, int64_t nt,
                  const int64_t *tgt, double *v, double *psi) {
    const or_t *o = (const or_t *)h;
    mode_t3 *modes;
    int64_t nm = half_modes(K, &modes);
    double complex *w = (double complex *)malloc(sizeof(double complex) * 3 * nm);
    omega_hat(o, K, nm, modes, w);
    double k0 = 2 * OR_PI / o->L;
    double complex *vh = (double complex *)malloc(sizeof(double complex) * 3 * nm);
    double complex *ph = (double complex *)malloc(sizeof(double complex) * 3 * nm);
    for (int64_t t = 0; t < nm; t++) {
        double k[3] = {k0 * modes[t].mx, k0 * modes[t].my, k0 * modes[t].mz};
        double k2 = dot3(k, k);
        double f = exp(-k2 / (4 * alpha * alpha)) / k2;
        double complex *wt = w + 3 * t;
        /* i k x w */
        vh[3 * t + 0] = I * (k[1] * wt[2] - k[2] * wt[1]) * f;
        vh[3 * t + 1] = I * (k[2] * wt[0] - k[0] * wt[2]) * f;
        vh[3 * t + 2] = I * (k[0] * wt[1] - k[1] * wt[0]) * f;
        for (int c = 0; c < 3; c++) ph[3 * t + c] = wt[c] * f;
    }
    int W = 2 * K + 1;
#pragma omp parallel
    {
        double complex *e = (double complex *)malloc(sizeof(double complex) * 3 * W);
#pragma omp for schedule(static)
        for (int64_t tt = 0; tt < nt; tt++) {
            const double *xi = o->x + 3 * tgt[tt];
            for (int c = 0; c < 3; c++)
                for (int m = -K; m <= K; m++)
                    e[c * W + m + K] = cexp(I * (k0 * m * xi[c]));
            double complex sv[3] = {0, 0, 0}, sp[3] = {0, 0, 0};
            for (int64_t t = 0; t < nm; t++) {
                double complex p = e[modes[t].mx + K] * e[W + modes[t].my + K] *
                                   e[2 * W + modes[t].mz + K];
                for (int c = 0; c < 3; c++) {
                    sv[c] += vh[3 * t + c] * p;
                    sp[c] += ph[3 * t + c] * p;
                }
            }
            for (int c = 0; c < 3; c++) {
                if (v) v[3 * tt + c] = 2.0 * creal(sv[c]);
                if (psi) psi[3 * tt + c] = 2.0 * creal(sp[c]);
            }
        }
        free(e);
    }
    free(modes); free(w); free(vh); free(ph);
}

/* Fourier coefficients of the vorticity, for direct tests of a spreading
 * step: out[(mz*(2K+1)+my+K)*(2K+1)+mx+K][3] over mz in [0,K] (complex as
 * re,im pairs), zero where the mode is not in the half space. */
void or_omega_hat(const void *h, int K, double *out) {
    const or_t *o = (const or_t *)h;
    mode_t3 *modes;
    int64_t nm = half_modes(K, &modes);
    double complex *w = (double complex *)malloc(sizeof(double complex) * 3 * nm);
    omega_hat(o, K, nm, modes, w);
    int W = 2 * K + 1;
    memset(out, 0, sizeof(double) * 2 * 3 * (size_t)W * W * (K + 1));
    for (int64_t t = 0; t < nm; t++) {
        size_t idx = ((size_t)modes[t].mz * W + modes[t].my + K) * W + modes[t].mx + K;
        for (int c = 0; c < 3; c++) {
            out[2 * (3 * idx + c)] = creal(w[3 * t + c]);
            out[2 * (3 * idx + c) + 1] = cimag(w[3 * t + c]);
        }
    }
    free(modes); free(w);
}

/* ------------------------------------------------------ brute force images */
/* Unsplit discrete Biot-Savart sum (alpha = 0) over the cubic shell of images
 * |n|_inf <= K, local segments excluded for n = 0 (eq:BS_on_vortex with the
 * lattice sum truncated; no local term). */
void or_brute_images(const void *h, int K, int64_t nt, const int64_t *tgt, double *v) {
    const or_t *o = (const or_t *)h;
    double L = o->L;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t], ip = prev_node(o, i);
        const double *xi = o->x + 3 * i;
        double acc[3] = {0, 0, 0};
        for (int nx = -K; nx <= K; nx++)
        for (int ny = -K; ny <= K; ny++)
        for (int nz = -K; nz <= K; nz++) {
            double part[3] = {0, 0, 0};
            for (int64_t q = 0; q < o->Nq; q++) {
                int64_t seg = q / o->Q;
                if (nx == 0 && ny == 0 && nz == 0 && (seg == i || seg == ip)) continue;
                double r[3] = {o->qx[3 * q] - xi[0] + nx * L, o->qx[3 * q + 1] - xi[1] + ny * L,
                               o->qx[3 * q + 2] - xi[2] + nz * L};
                double r2 = dot3(r, r), rr = sqrt(r2), cr[3];
                cross3(r, o->qc + 3 * q, cr);
                for (int c = 0; c < 3; c++) part[c] += cr[c] / (r2 * rr);
            }
            for (int c = 0; c < 3; c++) acc[c] += part[c];
        }
        for (int c = 0; c < 3; c++) v[3 * t + c] = acc[c] / (4 * OR_PI);
    }
}

/* ------------------------------------------------------------ diagnostics */
/* E = (1/2V) sum_l Gamma_l sum_j psi_j . sdot_j (dtau_{j-1} + dtau_j)/2
 * (eq:kinetic_energy_streamfunction, nodal trapezoid in tau). */
/* E = (1/2V) sum_l Gamma_l oint psi . ds (eq:kinetic_energy_streamfunction):
 * psi between the nodes is the spline through its nodal values on the
 * curve's own knots (cubic or quintic, as the curve), and the line integral
 * uses the curve's Q-point rule on every segment, so that
 * E = (1/2V) sum_q psi(tau_q) . q_q with the vector charges q_q. */
double or_energy(const void *h, const double *psi) {
    const or_t *o = (const or_t *)h;
    double V = o->L * o->L * o->L, e = 0.0;
    double *aux = (double *)calloc((size_t)(3 * o->N), sizeof(double));
    for (int64_t f = 0; f < o->nfil; f++) {
        if (o->order == 6) quintic_fit(o, f, psi, 0, aux);
        else cubic_fit(o, f, psi, 0, aux);
    }
    for (int64_t j = 0; j < o->N; j++)
        for (int i = 0; i < o->Q; i++) {
            double pv[3];
            spline_eval_data(o, psi, aux, j, o->gl_h[i] * o->dtau[j], 0, 0, pv);
            e += dot3(pv, o->qc + 3 * (j * o->Q + i));
        }
    free(aux);
    return e / (2 * V);
}

/* p = (1/2V) sum_q s_q x q_q (charges carry Gamma). */
void or_impulse(const void *h, double *p) {
    const or_t *o = (const or_t *)h;
    double V = o->L * o->L * o->L;
    p[0] = p[1] = p[2] = 0;
    for (int64_t q = 0; q < o->Nq; q++) {
        double c[3];
        cross3(o->qx + 3 * q, o->qc + 3 * q, c);
        for (int k = 0; k < 3; k++) p[k] += c[k];
    }
    for (int k = 0; k < 3; k++) p[k] /= 2 * V;
}

double or_length(const void *h) {
    const or_t *o = (const or_t *)h;
    double s = 0;
    for (int64_t j = 0; j < o->N; j++) s += o->ell[j];
    return s;
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* ------------------------------------------------------- near-singular */
/* Gauss-Kronrod 7/15 abscissae and weights on [-1,1] (QUADPACK's published
 * table).  Index 7 is the centre; odd indices 1,3,5 and 7 are the Gauss
 * points. */
static const double GK_X[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.0};
static const double GK_WK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double GK_WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

/* Full Biot-Savart kernel (Gamma/4pi)(s - x) x sdot/|s - x|^3 * dtau/du at
 * u in [0,1] of segment seg; xs is the target already shifted to the image of
 * the segment. */
static double ns_integrand(const or_t *o, int64_t seg, const double *xs, double u,
                           double *out) {
    double s[3], sd[3], r[3], c[3];
    double h = o->dtau[seg];
    seg_eval(o, seg, u * h, 0, s);
    seg_eval(o, seg, u * h, 1, sd);
    for (int k = 0; k < 3; k++) r[k] = s[k] - xs[k];
    double r2 = dot3(r, r), rr = sqrt(r2);
    cross3(r, sd, c);
    double g = o->gamma[o->fil[seg]] / (4 * OR_PI) * h / (r2 * rr);
    for (int k = 0; k < 3; k++) out[k] = c[k] * g;
    /* relative rounding noise of the value: r = s - x loses digits */
    return 2.220446049250313e-16 * (norm3(s) + norm3(xs)) / rr;
}

static void gk15(const or_t *o, int64_t seg, const double *xs, double a, double b,
                 double *rk, double *err, double *noise) {
    double m = 0.5 * (a + b), hw = 0.5 * (b - a);
    double sk[3] = {0, 0, 0}, sg[3] = {0, 0, 0}, f[3], sa = 0;
    for (int i = 0; i < 8; i++) {
        int ng = (i & 1) ? (i >> 1) : -1;        /* Gauss index or -1 */
        if (i == 7) ng = 3;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            if (i == 7 && sgn == 1) break;       /* centre once */
            double nz = ns_integrand(o, seg, xs, m + sgn * hw * GK_X[i], f);
            for (int k = 0; k < 3; k++) {
                sk[k] += GK_WK[i] * f[k];
                if (ng >= 0) sg[k] += GK_WG[ng] * f[k];
            }
            sa += GK_WK[i] * norm3(f) * (nz + 2.220446049250313e-16);
        }
    }
    double e = 0;
    for (int k = 0; k < 3; k++) {
        rk[k] = sk[k] * hw;
        double d = (sk[k] - sg[k]) * hw;
        e += d * d;
    }
    *err = sqrt(e);
    *noise = sa * hw;   /* integral of |F| times its relative noise */
}

/* Exact integral of the full kernel over segment seg (u in [0,1]) at target
 * x shifted by the image offset `shift` (x + shift is used), by adaptive
 * bisection: a piece [a,b] is accepted when its Kronrod-Gauss difference is
 * below tol * scale * (b - a), where scale is the integral of |kernel| over
 * the segment (so rounding of a cancelling sum cannot stall the test).
 * Returns the number of accepted pieces, negated if the piece budget ran
 * out before every piece met the tolerance. */
static void gk15_abs(const or_t *o, int64_t seg, const double *xs, double a,
                     double b, double *val) {
    double m = 0.5 * (a + b), hw = 0.5 * (b - a), s = 0, f[3];
    for (int i = 0; i < 8; i++)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            if (i == 7 && sgn == 1) break;
            ns_integrand(o, seg, xs, m + sgn * hw * GK_X[i], f);
            s += GK_WK[i] * norm3(f);
        }
    *val = s * hw;
}

int or_segment_integral(const void *h, int64_t seg, const double *x,
                        const double *shift, double tol, double *out) {
    const or_t *o = (const or_t *)h;
    double xs[3] = {x[0] + shift[0], x[1] + shift[1], x[2] + shift[2]};
    enum { MAXS = 256, MAXPIECES = 100000 };
    double sa[MAXS], sb[MAXS];
    int top, pieces = 0, ok = 1;
    /* scale: integral of |F| estimated on a uniform 64-piece split */
    double scale = 0.0;
    for (int k = 0; k < 64; k++) {
        double v;
        gk15_abs(o, seg, xs, k / 64.0, (k + 1) / 64.0, &v);
        scale += v;
    }
    double abstol = tol * scale;
    out[0] = out[1] = out[2] = 0;
    sa[0] = 0.0; sb[0] = 1.0; top = 1;
    while (top > 0) {
        top--;
        double a = sa[top], b = sb[top], r[3], e, ai;
        gk15(o, seg, xs, a, b, r, &e, &ai);
        /* accept at the requested accuracy, or at the rounding-noise floor
         * of the integrand on the piece (nothing finer is resolvable) */
        double lim = fmax(abstol * (b - a), 50.0 * ai);
        int last = (top + 2 >= MAXS) || (pieces >= MAXPIECES) || (b - a) < 1e-14;
        if (e <= lim || last) {
            if (e > lim) ok = 0;
            for (int k = 0; k < 3; k++) out[k] += r[k];
            pieces++;
        } else {
            double m = 0.5 * (a + b);
            sa[top] = m; sb[top] = b; top++;
            sa[top] = a; sb[top] = m; top++;
        }
    }
    return ok ? pieces : -pieces;
}

/* The Q-point sum the method uses for the same segment and target. */
void or_segment_qsum(const void *h, int64_t seg, const double *x,
                     const double *shift, double *out) {
    const or_t *o = (const or_t *)h;
    double xs[3] = {x[0] + shift[0], x[1] + shift[1], x[2] + shift[2]};
    out[0] = out[1] = out[2] = 0;
    for (int i = 0; i < o->Q; i++) {
        int64_t q = seg * o->Q + i;
        double r[3], c[3];
        for (int k = 0; k < 3; k++) r[k] = o->qx[3 * q + k] - xs[k];
        double r2 = dot3(r, r), rr = sqrt(r2);
        cross3(r, o->qc + 3 * q, c);
        for (int k = 0; k < 3; k++) out[k] += c[k] / (4 * OR_PI * r2 * rr);
    }
}

/* Biot-Savart integral of a straight segment A->B with circulation gamma at
 * x: (gamma/4pi) (r1 x r2)(p+q) / (p q (p q + r1.r2)), r1 = A-x, r2 = B-x,
 * p = |r1|, q = |r2| (textbook closed form of a straight vortex segment). */
void or_chord_integral(const double *A, const double *B, const double *x,
                       double gamma, double *out) {
    double r1[3], r2[3], c[3];
    for (int k = 0; k < 3; k++) { r1[k] = A[k] - x[k]; r2[k] = B[k] - x[k]; }
    double p = norm3(r1), q = norm3(r2);
    cross3(r1, r2, c);
    /* p q + r1.r2 loses digits when the target lies beside the segment
     * (r1.r2 < 0); there it equals |r1 x r2|^2 / (p q - r1.r2). */
    double dt = dot3(r1, r2);
    double den = (dt >= 0) ? p * q + dt : dot3(c, c) / (p * q - dt);
    double f = gamma / (4 * OR_PI) * (p + q) / (p * q * den);
    for (int k = 0; k < 3; k++) out[k] = c[k] * f;
}

/* Distance from x to the chord of segment seg and the image shift of x that
 * realises it (minimum image of the chord midpoint). */
static double chord_distance(const or_t *o, int64_t seg, const double *x, double *shift) {
    const double *A = o->x + 3 * seg;
    double B[3];
    seg_end(o, o->x, seg, 1, B);
    double m[3], e[3], r[3];
    for (int k = 0; k < 3; k++) {
        m[k] = 0.5 * (A[k] + B[k]);
        shift[k] = o->L * nearbyint((x[k] - m[k]) / o->L) * -1.0;
        e[k] = B[k] - A[k];
    }
    for (int k = 0; k < 3; k++) r[k] = x[k] + shift[k] - A[k];
    double t = dot3(r, e) / dot3(e, e);
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double d[3];
    for (int k = 0; k < 3; k++) d[k] = r[k] - t * e[k];
    return norm3(d);
}

/* Near-singular correction at target nodes: for every segment that is not
 * adjacent to the node and whose chord lies within eta * ell_seg of it,
 * add (exact segment integral) - (its Q-point sum).  nflag (optional)
 * receives the number of flagged segments per target. */
void or_ns_correction(const void *h, double eta, double tol, int64_t nt,
                      const int64_t *tgt, double *dv, int64_t *nflag) {
    const or_t *o = (const or_t *)h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t], ip = prev_node(o, i);
        const double *xi = o->x + 3 * i;
        double acc[3] = {0, 0, 0};
        int64_t cnt = 0;
        for (int64_t j = 0; j < o->N; j++) {
            if (j == i || j == ip) continue;
            double sh[3];
            double d = chord_distance(o, j, xi, sh);
            if (!(d < eta * o->ell[j])) continue;
            double ex[3], qs[3];
            or_segment_integral(o, j, xi, sh, tol, ex);
            or_segment_qsum(o, j, xi, sh, qs);
            for (int k = 0; k < 3; k++) acc[k] += ex[k] - qs[k];
            cnt++;
        }
        for (int k = 0; k < 3; k++) dv[3 * t + k] = acc[k];
        if (nflag) nflag[t] = cnt;
    }
}

/* ------------------------------------------------------------------ MLP */
/* Plain FP64 forward and backward pass of the 8-64-64-64-3 network with SiLU
 * activations, for checking device gradients.  Parameters are packed as
 * W1[64][8] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3];
 * loss = (1/2B) sum_b sum_c (y_bc - t_bc)^2. */
#define MLP_NP 9091
static const int MLP_DIMS[5] = {8, 64, 64, 64, 3};

int or_mlp_nparams(void) { return MLP_NP; }

static inline double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

static void mlp_layer_offsets(int *wo, int *bo) {
    int p = 0;
    for (int l = 0; l < 4; l++) {
        wo[l] = p; p += MLP_DIMS[l + 1] * MLP_DIMS[l];
        bo[l] = p; p += MLP_DIMS[l + 1];
    }
}

double or_mlp_loss_grad(const double *P, int64_t B, const double *X,
                        const double *T, double *Y, double *G) {
    int wo[4], bo[4];
    mlp_layer_offsets(wo, bo);
    if (G) memset(G, 0, sizeof(double) * MLP_NP);
    double loss = 0;
    for (int64_t b = 0; b < B; b++) {
        double z[4][64], hcur[5][64], dh[64], dz[64];
        for (int i = 0; i < 8; i++) hcur[0][i] = X[8 * b + i];
        for (int l = 0; l < 4; l++) {
            int ni = MLP_DIMS[l], no = MLP_DIMS[l + 1];
            for (int o = 0; o < no; o++) {
                double s = P[bo[l] + o];
                for (int i = 0; i < ni; i++) s += P[wo[l] + o * ni + i] * hcur[l][i];
                z[l][o] = s;
                hcur[l + 1][o] = (l < 3) ? s * sigm(s) : s;
            }
        }
        for (int c = 0; c < 3; c++) {
            if (Y) Y[3 * b + c] = hcur[4][c];
            if (T) {
                double d = hcur[4][c] - T[3 * b + c];
                loss += 0.5 * d * d / (double)B;
                dh[c] = d / (double)B;
            }
        }
        if (!G || !T) continue;
        for (int l = 3; l >= 0; l--) {
            int ni = MLP_DIMS[l], no = MLP_DIMS[l + 1];
            for (int o = 0; o < no; o++) {
                if (l < 3) {
                    double sg = sigm(z[l][o]);
                    dz[o] = dh[o] * sg * (1.0 + z[l][o] * (1.0 - sg));
                } else {
                    dz[o] = dh[o];
                }
            }
            double dprev[64];
            for (int i = 0; i < ni; i++) dprev[i] = 0;
            for (int o = 0; o < no; o++) {
                G[bo[l] + o] += dz[o];
                for (int i = 0; i < ni; i++) {
                    G[wo[l] + o * ni + i] += dz[o] * hcur[l][i];
                    dprev[i] += P[wo[l] + o * ni + i] * dz[o];
                }
            }
            for (int i = 0; i < ni; i++) dh[i] = dprev[i];
        }
    }
    return loss;
}
