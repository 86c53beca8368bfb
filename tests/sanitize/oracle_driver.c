/* Runs every entry point of the CPU oracle once on small filament sets read
 * from a binary file, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure only).
 *
 * Input file, native endian: int64 nsets, then per set
 *   int64 nfil, int64 order, int64 has_periods, int64 offsets[nfil + 1],
 *   double xyz[N][3], double gamma[nfil], double L, a, delta,
 *   int64 periods[nfil][3] (if has_periods)
 * Prints one checksum line per set. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void *or_new(int64_t nfil, const int64_t *off, const double *xyz, const double *gamma, double L,
             double a, double delta, int Q, int order, const int64_t *periods);
void or_free(void *h);
int64_t or_nquad(const void *h);
void or_get_quad(const void *h, double *pos, double *deriv, double *charge);
void or_get_nodes(const void *h, double *tau, double *dtau, double *sdot, double *sddot,
                  double *ell);
void or_spline_eval(const void *h, int64_t seg, double u, int deriv, double *out);
void or_local(const void *h, int64_t nt, const int64_t *tgt, double *v, double *psi);
void or_local_sub(const void *h, double eps, int64_t nt, const int64_t *tgt, double *v,
                  double *psi);
void or_shortrange(const void *h, double alpha, double rc, int64_t nt, const int64_t *tgt,
                   double *v, double *psi);
void or_selfcorr(const void *h, double alpha, int64_t nt, const int64_t *tgt, double *v,
                 double *psi);
void or_longrange(const void *h, double alpha, int K, int64_t nt, const int64_t *tgt, double *v,
                  double *psi);
void or_omega_hat(const void *h, int K, double *out);
void or_brute_images(const void *h, int K, int64_t nt, const int64_t *tgt, double *v);
double or_energy(const void *h, const double *psi);
void or_impulse(const void *h, double *p);
double or_length(const void *h);
int or_segment_integral(const void *h, int64_t seg, const double *x, const double *shift,
                        double tol, double *out);
void or_segment_qsum(const void *h, int64_t seg, const double *x, const double *shift,
                     double *out);
void or_chord_integral(const double *A, const double *B, const double *x, double gamma,
                       double *out);
void or_ns_correction(const void *h, double eta, double tol, int64_t nt, const int64_t *tgt,
                      double *dv, int64_t *nflag);
int or_gl_rule(int Q, double *h, double *w);
void or_cyclic_tridiag(int64_t n, const double *a, const double *b, const double *c, double *x);
int or_mlp_nparams(void);
double or_mlp_loss_grad(const double *P, int64_t B, const double *X, const double *T, double *Y,
                        double *G);
double or_g_lr(double x);
double or_g_sr(double x);

static double sum_abs(const double *v, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += fabs(v[i]);
    return s;
}

static int64_t rd_i(FILE *f) {
    int64_t v;
    if (fread(&v, sizeof v, 1, f) != 1) exit(2);
    return v;
}

static void rd_d(FILE *f, double *p, size_t n) {
    if (fread(p, sizeof *p, n, f) != n) exit(2);
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    const int64_t nsets = rd_i(f);
    for (int64_t s = 0; s < nsets; s++) {
        const int64_t nfil = rd_i(f), order = rd_i(f), hasp = rd_i(f);
        int64_t *off = malloc(sizeof(int64_t) * (nfil + 1));
        for (int64_t i = 0; i <= nfil; i++) off[i] = rd_i(f);
        const int64_t N = off[nfil];
        double *xyz = malloc(sizeof(double) * 3 * N), *gam = malloc(sizeof(double) * nfil);
        rd_d(f, xyz, 3 * N);
        rd_d(f, gam, nfil);
        double prm[3];
        rd_d(f, prm, 3);
        int64_t *per = NULL;
        if (hasp) {
            per = malloc(sizeof(int64_t) * 3 * nfil);
            for (int64_t i = 0; i < 3 * nfil; i++) per[i] = rd_i(f);
        }
        for (int Q = 1; Q <= 4; Q++) {
            void *h = or_new(nfil, off, xyz, gam, prm[0], prm[1], prm[2], Q, (int)order, per);
            if (!h) { printf("set %lld: or_new failed\n", (long long)s); return 1; }
            const int64_t Nq = or_nquad(h);
            double *qa = malloc(sizeof(double) * 3 * Nq), *qb = malloc(sizeof(double) * 3 * Nq),
                   *qc = malloc(sizeof(double) * 3 * Nq);
            or_get_quad(h, qa, qb, qc);
            double *nd = malloc(sizeof(double) * 9 * N);
            or_get_nodes(h, nd, nd + N, nd + 2 * N, nd + 5 * N, nd + 8 * N);
            int64_t *tg = malloc(sizeof(int64_t) * N);
            for (int64_t i = 0; i < N; i++) tg[i] = i;
            double *v = calloc(3 * N, sizeof(double)), *p = calloc(3 * N, sizeof(double));
            double *w = calloc(3 * N, sizeof(double)), *e = calloc(3 * N, sizeof(double));
            const double L = prm[0], alpha = 6.0 / (L / 2), rc = L / 2;
            or_local(h, N, tg, v, p);
            or_local_sub(h, 0.1, N, tg, w, e);
            or_shortrange(h, alpha, rc, N, tg, w, e);
            or_shortrange(h, 0.0, L, N, tg, w, NULL);
            or_selfcorr(h, alpha, N, tg, w, e);
            or_longrange(h, alpha, 6, N, tg, w, e);
            or_longrange(h, alpha, 6, N, tg, w, NULL);
            const int K = 3, W = 2 * K + 1;
            double *om = malloc(sizeof(double) * 6 * W * W * (K + 1));
            or_omega_hat(h, K, om);
            or_brute_images(h, 1, N < 8 ? N : 8, tg, w);
            double imp[3], seg[3], x0[3] = {0.01, 0.02, 0.03}, sh[3] = {0, 0, 0};
            or_impulse(h, imp);
            double acc = or_energy(h, e) + or_length(h) + sum_abs(imp, 3);
            for (int64_t j = 0; j < (N < 4 ? N : 4); j++) {
                double x1[3] = {xyz[3 * j] + 1e-3, xyz[3 * j + 1], xyz[3 * j + 2] - 2e-3};
                or_spline_eval(h, j, 0.3, 2, seg);
                acc += sum_abs(seg, 3);
                or_segment_integral(h, (j + 2) % N, x1, sh, 1e-12, seg);
                acc += sum_abs(seg, 3);
                or_segment_qsum(h, (j + 2) % N, x0, sh, seg);
                acc += sum_abs(seg, 3);
            }
            or_ns_correction(h, 1.0, 1e-12, N, tg, w, NULL);
            int64_t *cnt = malloc(sizeof(int64_t) * N);
            or_ns_correction(h, 0.5, 1e-12, N, tg, e, cnt);
            acc += sum_abs(v, 3 * N) + sum_abs(p, 3 * N) + sum_abs(w, 3 * N) + sum_abs(e, 3 * N) +
                   sum_abs(qa, 3 * Nq) + sum_abs(qb, 3 * Nq) + sum_abs(qc, 3 * Nq) +
                   sum_abs(nd, 9 * N) + sum_abs(om, 6 * W * W * (K + 1));
            printf("set %lld Q %d: %.6e\n", (long long)s, Q, acc);
            free(qa); free(qb); free(qc); free(nd); free(tg); free(v); free(p); free(w); free(e);
            free(om); free(cnt);
            or_free(h);
        }
        free(off); free(xyz); free(gam); free(per);
    }
    fclose(f);
    /* helpers with no filament set */
    double gh[8], gw[8], out[3], A[3] = {0, 0, 0}, Bp[3] = {1, 0, 0}, x[3] = {0.5, 0.1, 0};
    for (int Q = 1; Q <= 4; Q++) or_gl_rule(Q, gh, gw);
    or_chord_integral(A, Bp, x, 1.0, out);
    double a[7], b[7], c[7], r[7];
    for (int i = 0; i < 7; i++) { a[i] = 1; b[i] = 4; c[i] = 1; r[i] = i; }
    or_cyclic_tridiag(7, a, b, c, r);
    const int np = or_mlp_nparams();
    double *P = calloc(np, sizeof(double)), *G = calloc(np, sizeof(double));
    for (int i = 0; i < np; i++) P[i] = 0.01 * ((i * 37) % 11 - 5);
    double X[5 * 8], T[5 * 3], Y[5 * 3];
    for (int i = 0; i < 40; i++) X[i] = 0.1 * (i % 7) - 0.3;
    for (int i = 0; i < 15; i++) T[i] = 0.2 * (i % 5);
    const double loss = or_mlp_loss_grad(P, 5, X, T, Y, G);
    printf("helpers: %.6e %.6e %.6e %.6e\n", out[0] + out[1] + out[2] + r[3], loss,
           or_g_lr(0.3) + or_g_sr(0.3), sum_abs(G, np));
    free(P); free(G);
    return 0;
}
