// Filament geometry on the device, all in float64:
//   chord-length parametrisation and the periodic cubic spline (App. B),
//   quadrature points and vector charges (Sec. 2.7 and Sec. 3.3,
//   eq:line_integral_quadrature, eq:vorticity_fourier_coefs),
//   local terms (eq:BS_local, eq:streamfunction_local) and the long-range
//   self corrections (eq:velocity_longrange_self,
//   eq:streamfunction_longrange_self).
//
// Spline form used here: cubic Hermite segments whose node slopes D_j solve
// the C2 conditions  h_j D_{j-1} + 2 (h_{j-1} + h_j) D_j + h_{j-1} D_{j+1}
// = 3 (h_j d_{j-1} + h_{j-1} d_j),  d_j = (s_{j+1} - s_j) / h_j, indices
// periodic.  The periodic interpolating cubic spline on given knots is
// unique, so this is the same curve as the paper's B-spline form.  The
// cyclic tridiagonal system is solved by parallel cyclic reduction, one
// workgroup per filament: each step eliminates the neighbours at distance
// d = 2^s, squaring the off-diagonal to diagonal ratio (<= 1/2 here), so
// after 7 steps they are below 1e-19 and D_i = r_i / b_i.
#include "bs_internal.h"

namespace bs {

__device__ __forceinline__ int next_node(const int *off, const int *fil, int j) {
    int f = fil[j];
    return (j + 1 < off[f + 1]) ? j + 1 : off[f];
}
__device__ __forceinline__ int prev_node(const int *off, const int *fil, int j) {
    int f = fil[j];
    return (j > off[f]) ? j - 1 : off[f + 1] - 1;
}

// ------------------------------------------------------------- chord lengths
// Chord lengths from the caller's node positions, which are copied into the
// plan's own array on the way (xs may alias xd); thread f < nfil also copies
// filament f's circulation.
__global__ void k_chord(int N, int nfil, const double *xs, double *xd,
                        const double *__restrict__ gs, double *__restrict__ gd,
                        const int *__restrict__ off, const int *__restrict__ fil,
                        double *__restrict__ dtau, int *__restrict__ status) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nfil) gd[j] = gs[j];
    if (j >= N) return;
    int jn = next_node(off, fil, j);
    const double x0 = xs[3 * j], x1 = xs[3 * j + 1], x2 = xs[3 * j + 2];
    double dx = xs[3 * jn] - x0, dy = xs[3 * jn + 1] - x1, dz = xs[3 * jn + 2] - x2;
    double h = sqrt(dx * dx + dy * dy + dz * dz);
    bool ok = isfinite(x0) && isfinite(x1) && isfinite(x2) && isfinite(h) && h > 0.0;
    if (!ok) atomicOr(status, 1);
    dtau[j] = ok ? h : 1.0;
    xd[3 * j] = x0; xd[3 * j + 1] = x1; xd[3 * j + 2] = x2;
}

// ------------------------------------------------------------- spline (PCR)
constexpr int kPcrSteps = 7;
constexpr int kPcrLds = 512;   // nodes per filament solved in LDS

struct PcrArrays {
    double *a, *b, *c, *r;     // r holds 3 components: r[3*k + comp]
};

__device__ void pcr_solve(int n, PcrArrays A, PcrArrays B) {
    // A holds the system on entry; ping-pong with B; the solution of the
    // final step is left in whichever holds the last result.
    int d = 1;
    PcrArrays src = A, dst = B;
    for (int s = 0; s < kPcrSteps; s++) {
        int dm = d % n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int im = i - dm; if (im < 0) im += n;
            int ip = i + dm; if (ip >= n) ip -= n;
            double k1 = src.a[i] / src.b[im];
            double k2 = src.c[i] / src.b[ip];
            dst.a[i] = -k1 * src.a[im];
            dst.c[i] = -k2 * src.c[ip];
            dst.b[i] = src.b[i] - k1 * src.c[im] - k2 * src.a[ip];
#pragma unroll
            for (int q = 0; q < 3; q++)
                dst.r[3 * i + q] = src.r[3 * i + q] - k1 * src.r[3 * im + q] - k2 * src.r[3 * ip + q];
        }
        __syncthreads();
        PcrArrays t = src; src = dst; dst = t;
        d *= 2;
    }
    // after an odd number of steps the result is in B
}

__global__ void k_spline(int nfil, const int *__restrict__ off, const double *__restrict__ x,
                         const double *__restrict__ dtau, double *__restrict__ D,
                         double *__restrict__ gscratch) {
    __shared__ double lds[2 * 6 * kPcrLds];
    int f = blockIdx.x;
    if (f >= nfil) return;
    int b0 = off[f], n = off[f + 1] - off[f];
    double *base;
    if (n <= kPcrLds) base = lds;
    else base = gscratch + (size_t)12 * b0;   // 12 doubles per node
    int stride = (n <= kPcrLds) ? kPcrLds : n;
    PcrArrays A{base, base + stride, base + 2 * stride, base + 3 * stride};
    PcrArrays B{base + 6 * stride, base + 7 * stride, base + 8 * stride, base + 9 * stride};
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        int km = (k == 0) ? n - 1 : k - 1, kp = (k + 1 == n) ? 0 : k + 1;
        double hm = dtau[b0 + km], hk = dtau[b0 + k];
        A.a[k] = hk;
        A.b[k] = 2.0 * (hm + hk);
        A.c[k] = hm;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            double sm = x[3 * (b0 + km) + q], s0 = x[3 * (b0 + k) + q], sp = x[3 * (b0 + kp) + q];
            A.r[3 * k + q] = 3.0 * (hk * (s0 - sm) / hm + hm * (sp - s0) / hk);
        }
    }
    __syncthreads();
    pcr_solve(n, A, B);
    PcrArrays R = (kPcrSteps & 1) ? B : A;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 3; q++) D[3 * (b0 + k) + q] = R.r[3 * k + q] / R.b[k];
    }
}

// --------------------------------------------------------- segment geometry
struct GLArgs {
    double h[kMaxQ];
    double w[kMaxQ];
};

// Hermite segment j: s(u) = c0 + c1 u + c2 u^2 + c3 u^3, u in [0,1],
// tau = tau_j + u h; ds/dtau = s'(u)/h.
__global__ void k_geometry(int N, int Q, GLArgs gl, const double *__restrict__ x,
                           const int *__restrict__ off, const int *__restrict__ fil,
                           const double *__restrict__ gamma, const double *__restrict__ dtau,
                           const double *__restrict__ D, double *__restrict__ qpos,
                           double *__restrict__ qchg, double *__restrict__ sdd,
                           double *__restrict__ ell) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    int jn = next_node(off, fil, j);
    double h = dtau[j], g = gamma[fil[j]];
    double c0[3], c1[3], c2[3], c3[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        double s0 = x[3 * j + q], s1 = x[3 * jn + q];
        double d0 = h * D[3 * j + q], d1 = h * D[3 * jn + q];
        c0[q] = s0;
        c1[q] = d0;
        c2[q] = 3.0 * (s1 - s0) - 2.0 * d0 - d1;
        c3[q] = 2.0 * (s0 - s1) + d0 + d1;
        sdd[3 * j + q] = 2.0 * c2[q] / (h * h);
    }
    double len = 0.0;
    for (int i = 0; i < Q; i++) {
        double u = gl.h[i];
        double der[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            qpos[3 * (j * Q + i) + q] = c0[q] + u * (c1[q] + u * (c2[q] + u * c3[q]));
            der[q] = (c1[q] + u * (2.0 * c2[q] + 3.0 * u * c3[q])) / h;
            qchg[3 * (j * Q + i) + q] = g * gl.w[i] * h * der[q];
        }
        len += gl.w[i] * h * sqrt(der[0] * der[0] + der[1] * der[1] + der[2] * der[2]);
    }
    ell[j] = len;
}

// -------------------------------------------------------- local + self terms
// g_lr(x) = erf(x) - (2x/sqrt(pi)) exp(-x^2) (eq:ewald_derivative_weight_
// functions).  Below x = 0.5 the two terms cancel; there g_lr(x)/x^3 is
// summed from its Taylor series, coefficient n (n >= 1) of x^(2n-2) being
// (2/sqrt(pi)) (-1)^(n+1) 2n / (n! (2n+1)).
__host__ __device__ constexpr double glr_coef(int n) {
    double f = 1.0;
    for (int k = 1; k <= n; k++) f *= k;
    return ((n & 1) ? 2.0 : -2.0) * n / (f * (2.0 * n + 1.0));
}

__device__ __forceinline__ double glr_over_x3(double x) {
    if (x < 0.5) {
        constexpr double c[15] = {0.0,           glr_coef(1),  glr_coef(2),  glr_coef(3),
                                  glr_coef(4),   glr_coef(5),  glr_coef(6),  glr_coef(7),
                                  glr_coef(8),   glr_coef(9),  glr_coef(10), glr_coef(11),
                                  glr_coef(12),  glr_coef(13), glr_coef(14)};
        double x2 = x * x, acc = 0.0;
#pragma unroll
        for (int n = 14; n >= 1; n--) acc = acc * x2 + c[n];
        return acc * 1.12837916709551257389615890312154517;   // 2/sqrt(pi)
    }
    return (erf(x) - 1.12837916709551257389615890312154517 * x * exp(-x * x)) / (x * x * x);
}

__device__ __forceinline__ double erf_over_x(double x) {
    if (x < 1e-8) return 1.12837916709551257389615890312154517;
    return erf(x) / x;
}

__global__ void k_local_self(int N, int Q, int mode, double sign, double a, double delta,
                             double alpha, const double *__restrict__ x,
                             const int *__restrict__ off, const int *__restrict__ fil,
                             const double *__restrict__ gamma, const double *__restrict__ D,
                             const double *__restrict__ sdd, const double *__restrict__ ell,
                             const double *__restrict__ qpos, const double *__restrict__ qchg,
                             double *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double inv4pi = 1.0 / (4.0 * kPi);
    int ip = prev_node(off, fil, i);
    double g = gamma[fil[i]];
    bool psi = (mode & LS_PSI) != 0;
    double acc[3] = {0.0, 0.0, 0.0};
    if (mode & LS_VLOCAL) {
        double sd[3] = {D[3 * i], D[3 * i + 1], D[3 * i + 2]};
        double sn = sqrt(sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]);
        double lg = log(2.0 * sqrt(ell[ip] * ell[i]) / a);
        if (!psi) {
            double s2[3] = {sdd[3 * i], sdd[3 * i + 1], sdd[3 * i + 2]};
            double b[3] = {sd[1] * s2[2] - sd[2] * s2[1], sd[2] * s2[0] - sd[0] * s2[2],
                           sd[0] * s2[1] - sd[1] * s2[0]};
            double f = g * inv4pi * (lg - delta) / (sn * sn * sn);
            for (int q = 0; q < 3; q++) acc[q] += f * b[q];
        } else {
            double f = g / (2.0 * kPi) * (lg - (delta - 1.0)) / sn;
            for (int q = 0; q < 3; q++) acc[q] += f * sd[q];
        }
    }
    if (mode & LS_VSELF) {
        double self[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < Q; k++) {
                int qi = (s == 0 ? ip : i) * Q + k;
                double r[3], c[3];
                for (int q = 0; q < 3; q++) r[q] = qpos[3 * qi + q] - x[3 * i + q];
                const double *ch = qchg + 3 * qi;
                double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                if (!psi) {
                    c[0] = r[1] * ch[2] - r[2] * ch[1];
                    c[1] = r[2] * ch[0] - r[0] * ch[2];
                    c[2] = r[0] * ch[1] - r[1] * ch[0];
                    double f = alpha * alpha * alpha * glr_over_x3(alpha * rr);
                    for (int q = 0; q < 3; q++) self[q] += f * c[q];
                } else {
                    double f = alpha * erf_over_x(alpha * rr);
                    for (int q = 0; q < 3; q++) self[q] += f * ch[q];
                }
            }
        double sg = (mode & LS_VLOCAL) ? -1.0 : 1.0;   // local - self
        for (int q = 0; q < 3; q++) acc[q] += sg * inv4pi * self[q];
    }
    for (int q = 0; q < 3; q++) {
        if (mode & LS_ASSIGN) out[3 * i + q] = sign * acc[q];
        else out[3 * i + q] += sign * acc[q];
    }
}

// ------------------------------------------------------------------ launch
static inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

void launch_chord(bs_plan_t p, const double *xyz, const double *gamma) {
    if (p->N == 0) return;
    const int64_t items = p->N > p->nfil ? p->N : p->nfil;
    hipLaunchKernelGGL(k_chord, dim3(blocks_for(items, 256)), dim3(256), 0, p->stream, (int)p->N,
                       (int)p->nfil, xyz, (double *)p->d_x.p, gamma, (double *)p->d_gamma.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (double *)p->d_dtau.p, (int *)p->d_status.p);
}

void launch_spline(bs_plan_t p) {
    hipLaunchKernelGGL(k_spline, dim3((unsigned)p->nfil), dim3(128), 0, p->stream, (int)p->nfil,
                       (const int *)p->d_off.p, (const double *)p->d_x.p,
                       (const double *)p->d_dtau.p, (double *)p->d_D.p,
                       (double *)p->spline_tmp.p);
}

void launch_geometry(bs_plan_t p) {
    GLRule r = gl_rule(p->Q);
    GLArgs g;
    for (int i = 0; i < kMaxQ; i++) { g.h[i] = r.h[i]; g.w[i] = r.w[i]; }
    hipLaunchKernelGGL(k_geometry, dim3(blocks_for(p->N, 256)), dim3(256), 0, p->stream,
                       (int)p->N, p->Q, g, (const double *)p->d_x.p, (const int *)p->d_off.p,
                       (const int *)p->d_fil.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_dtau.p, (const double *)p->d_D.p,
                       (double *)p->d_qpos.p, (double *)p->d_qchg.p, (double *)p->d_sdd.p,
                       (double *)p->d_ell.p);
}

void launch_local_self(bs_plan_t p, int mode, double sign, double *out) {
    hipLaunchKernelGGL(k_local_self, dim3(blocks_for(p->N, 256)), dim3(256), 0, p->stream,
                       (int)p->N, p->Q, mode, sign, p->prm.a, p->prm.delta, p->prm.alpha,
                       (const double *)p->d_x.p, (const int *)p->d_off.p,
                       (const int *)p->d_fil.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_D.p, (const double *)p->d_sdd.p,
                       (const double *)p->d_ell.p, (const double *)p->d_qpos.p,
                       (const double *)p->d_qchg.p, out);
}

}  // namespace bs
