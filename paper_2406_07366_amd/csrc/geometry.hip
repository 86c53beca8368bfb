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
// d = 2^s, which shrinks the off-diagonal to diagonal ratio from 1/2 to
// below rounding in kPcrSteps = 6 steps (the bound is below), after which
// D_i = r_i / b_i.
//
// Quintic splines (App. B, k = 6) use the same idea with quintic Hermite
// segments: node values s_i, slopes D_i and second derivatives S_i; C3 and C4
// continuity at every node give a cyclic block-tridiagonal system in
// X_i = (D_i, S_i) with 2x2 blocks, solved by block parallel cyclic
// reduction (the interpolating periodic quintic spline on given knots is
// unique, so this is the paper's curve).
#include "bs_internal.h"
#include "bs_device.h"

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
// Chord lengths of filament f from the caller's node positions, which are
// copied into the plan's own array on the way (xs may alias xd); also the
// plan's copy of the filament's circulation and the end node of every
// segment in the segment's own frame (xn).  An infinite filament
// (s(tau + T) = s(tau) + n L, Sec. 2.1) has its period shift n L in shift;
// its last segment ends at the first node plus that shift.  shift NULL: all
// filaments closed.  Non-finite positions and zero-length segments set bit 0
// of the status word (their chord is taken as 1 so that the rest stays
// finite).
__device__ void chord_fil(int f, int b0, int n, const double *xs, double *xd,
                          double *__restrict__ xn, const double *__restrict__ shift,
                          const double *__restrict__ gs, double *__restrict__ gd,
                          double *__restrict__ dtau, int *__restrict__ status) {
    if (threadIdx.x == 0) gd[f] = gs[f];
    double sh[3] = {0.0, 0.0, 0.0};
    if (shift)
        for (int q = 0; q < 3; q++) sh[q] = shift[3 * f + q];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const bool last = k + 1 == n;
        const int j = b0 + k, jn = last ? b0 : j + 1;
        const double x0 = xs[3 * j], x1 = xs[3 * j + 1], x2 = xs[3 * j + 2];
        const double e0 = last ? xs[3 * jn] + sh[0] : xs[3 * jn];
        const double e1 = last ? xs[3 * jn + 1] + sh[1] : xs[3 * jn + 1];
        const double e2 = last ? xs[3 * jn + 2] + sh[2] : xs[3 * jn + 2];
        const double dx = e0 - x0, dy = e1 - x1, dz = e2 - x2;
        const double h = sqrt(dx * dx + dy * dy + dz * dz);
        const bool ok = isfinite(x0) && isfinite(x1) && isfinite(x2) && isfinite(h) && h > 0.0;
        if (!ok) atomicOr(status, 1);
        dtau[j] = ok ? h : 1.0;
        xn[3 * j] = e0; xn[3 * j + 1] = e1; xn[3 * j + 2] = e2;
        xd[3 * j] = x0; xd[3 * j + 1] = x1; xd[3 * j + 2] = x2;
    }
}

// ------------------------------------------------------------- spline (PCR)
// Every row of the spline systems has |a| + |c| = |b| / 2, and a reduction
// step maps the ratio l = max (|a| + |c|) / |b| to at most l^2 / (1 - l^2):
// 1/2, 1/3, 1/8, 1/63, 2.5e-4, 6.3e-8, 4e-15 after six steps (measured
// worst case over node spacings 3000:1, 1e-37), whatever n, so the
// couplings left after six steps lie below rounding and x = r / b.
constexpr int kPcrSteps = 6;

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
    // the last step wrote B if kPcrSteps is odd, A if it is even
}

// slopes D of the cubic spline through the nodal data x of one filament
// (nodes b0 .. b0+n-1); xn: end node of each segment in its own frame, for
// positions (NULL for periodic data such as the streamfunction); the whole
// workgroup takes part
__device__ void spline_cubic_fil(int b0, int n, const double *__restrict__ x,
                                 const double *__restrict__ xn,
                                 const double *__restrict__ dtau, double *__restrict__ D,
                                 double *__restrict__ gscratch) {
    __shared__ double lds[2 * 6 * kPcrLds];
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
            const double s0 = x[3 * (b0 + k) + q], sm = x[3 * (b0 + km) + q];
            const double dm = (xn ? xn[3 * (b0 + km) + q] : s0) - sm;
            const double dp = (xn ? xn[3 * (b0 + k) + q] : x[3 * (b0 + kp) + q]) - s0;
            A.r[3 * k + q] = 3.0 * (hk * dm / hm + hm * dp / hk);
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

__global__ void k_spline(int nfil, const int *__restrict__ off, const double *__restrict__ x,
                         const double *__restrict__ xn, const double *__restrict__ dtau,
                         double *__restrict__ D, double *__restrict__ gscratch) {
    const int f = blockIdx.x;
    if (f >= nfil) return;
    spline_cubic_fil(off[f], off[f + 1] - off[f], x, xn, dtau, D, gscratch);
}

// ------------------------------------------------ quintic spline (block PCR)
// Rows of node i (h- = h_{i-1}, h+ = h_i), the C3 condition scaled by 1/3
// and the C4 condition by -1/12:
//   -8/h-^2 D_{i-1} - 1/h- S_{i-1} + 12 (1/h+^2 - 1/h-^2) D_i
//     + 3 (1/h- + 1/h+) S_i + 8/h+^2 D_{i+1} - 1/h+ S_{i+1}
//     = 20 [(s_{i+1} - s_i)/h+^3 - (s_i - s_{i-1})/h-^3]
//   14/h-^3 D_{i-1} + 2/h-^2 S_{i-1} + 16 (1/h-^3 + 1/h+^3) D_i
//     - 3 (1/h-^2 - 1/h+^2) S_i + 14/h+^3 D_{i+1} - 2/h+^2 S_{i+1}
//     = 30 [(s_i - s_{i-1})/h-^4 + (s_{i+1} - s_i)/h+^4]
// The diagonal block has det = -12 (1/h- + 1/h+)^4, never zero.  The
// influence of a node decays by about 0.43 per node (the quintic spline's
// cardinal function), so after 8 doubling steps the couplings left are
// below 0.43^256.  At distance n/2 of a power-of-two n both neighbours are
// the same node and their two couplings are merged.
constexpr int kPcr5Steps = 8;

struct Blk {
    double L[4], M[4], U[4], R[6];   // 2x2 blocks row-major; R[row * 3 + comp]
};

__device__ __forceinline__ void inv2(const double *A, double *B) {
    const double id = 1.0 / (A[0] * A[3] - A[1] * A[2]);
    B[0] = A[3] * id;
    B[1] = -A[1] * id;
    B[2] = -A[2] * id;
    B[3] = A[0] * id;
}
__device__ __forceinline__ void mul2(const double *A, const double *B, double *C) {
    C[0] = A[0] * B[0] + A[1] * B[2];
    C[1] = A[0] * B[1] + A[1] * B[3];
    C[2] = A[2] * B[0] + A[3] * B[2];
    C[3] = A[2] * B[1] + A[3] * B[3];
}
// C -= A B (2x2)
__device__ __forceinline__ void sub_mul2(const double *A, const double *B, double *C) {
    double t[4];
    mul2(A, B, t);
    for (int k = 0; k < 4; k++) C[k] -= t[k];
}
// R -= K V (K 2x2, V 2x3)
__device__ __forceinline__ void sub_mulR(const double *K, const double *V, double *R) {
    for (int r = 0; r < 2; r++)
        for (int q = 0; q < 3; q++) R[3 * r + q] -= K[2 * r] * V[q] + K[2 * r + 1] * V[3 + q];
}

// slopes D and second derivatives S of the quintic spline through the nodal
// data x of one filament; the whole workgroup takes part
__device__ void spline_quintic_fil(int b0, int n, const double *__restrict__ x,
                                   const double *__restrict__ xn,
                                   const double *__restrict__ dtau, double *__restrict__ D,
                                   double *__restrict__ S, double *__restrict__ gscratch) {
    __shared__ Blk lds[2 * kPcr5Lds];
    Blk *src, *dst;
    if (n <= kPcr5Lds) {
        src = lds;
        dst = lds + kPcr5Lds;
    } else {
        src = (Blk *)(gscratch + (size_t)36 * b0);   // 2 x 18 doubles per node
        dst = src + n;
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int km = (k == 0) ? n - 1 : k - 1, kp = (k + 1 == n) ? 0 : k + 1;
        const double hm = dtau[b0 + km], hp = dtau[b0 + k];
        const double im1 = 1.0 / hm, ip1 = 1.0 / hp;
        const double im2 = im1 * im1, ip2 = ip1 * ip1, im3 = im2 * im1, ip3 = ip2 * ip1;
        Blk &e = src[k];
        e.L[0] = -8.0 * im2;  e.L[1] = -im1;
        e.L[2] = 14.0 * im3;  e.L[3] = 2.0 * im2;
        e.M[0] = 12.0 * (ip2 - im2);   e.M[1] = 3.0 * (im1 + ip1);
        e.M[2] = 16.0 * (im3 + ip3);   e.M[3] = -3.0 * (im2 - ip2);
        e.U[0] = 8.0 * ip2;   e.U[1] = -ip1;
        e.U[2] = 14.0 * ip3;  e.U[3] = -2.0 * ip2;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const double s0 = x[3 * (b0 + k) + q], sm = x[3 * (b0 + km) + q];
            const double dm = (xn ? xn[3 * (b0 + km) + q] : s0) - sm;
            const double dp = (xn ? xn[3 * (b0 + k) + q] : x[3 * (b0 + kp) + q]) - s0;
            e.R[q] = 20.0 * (dp * ip3 - dm * im3);
            e.R[3 + q] = 30.0 * (dm * im3 * im1 + dp * ip3 * ip1);
        }
    }
    __syncthreads();
    int d = 1;
    for (int st = 0; st < kPcr5Steps; st++) {
        const int dm = d % n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int im = i - dm; if (im < 0) im += n;
            int ip = i + dm; if (ip >= n) ip -= n;
            const Blk &e = src[i];
            Blk &o = dst[i];
            double Mi[4], K[4];
            for (int k = 0; k < 4; k++) o.M[k] = e.M[k];
            for (int k = 0; k < 6; k++) o.R[k] = e.R[k];
            if (2 * dm == n) {
                // both neighbours are node ip: one coupling L_i + U_i
                double Ci[4], Cj[4];
                for (int k = 0; k < 4; k++) {
                    Ci[k] = e.L[k] + e.U[k];
                    Cj[k] = src[ip].L[k] + src[ip].U[k];
                }
                inv2(src[ip].M, Mi);
                mul2(Ci, Mi, K);
                sub_mul2(K, Cj, o.M);
                sub_mulR(K, src[ip].R, o.R);
                for (int k = 0; k < 4; k++) o.L[k] = o.U[k] = 0.0;
            } else {
                inv2(src[im].M, Mi);
                mul2(e.L, Mi, K);             // K1 = L_i M_im^-1
                mul2(K, src[im].L, o.L);
                for (int k = 0; k < 4; k++) o.L[k] = -o.L[k];
                sub_mul2(K, src[im].U, o.M);
                sub_mulR(K, src[im].R, o.R);
                inv2(src[ip].M, Mi);
                mul2(e.U, Mi, K);             // K2 = U_i M_ip^-1
                mul2(K, src[ip].U, o.U);
                for (int k = 0; k < 4; k++) o.U[k] = -o.U[k];
                sub_mul2(K, src[ip].L, o.M);
                sub_mulR(K, src[ip].R, o.R);
            }
        }
        __syncthreads();
        Blk *t = src; src = dst; dst = t;
        d *= 2;
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        double Mi[4];
        inv2(src[k].M, Mi);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const double r0 = src[k].R[q], r1 = src[k].R[3 + q];
            D[3 * (b0 + k) + q] = Mi[0] * r0 + Mi[1] * r1;
            S[3 * (b0 + k) + q] = Mi[2] * r0 + Mi[3] * r1;
        }
    }
}

__global__ void k_spline5(int nfil, const int *__restrict__ off, const double *__restrict__ x,
                          const double *__restrict__ xn, const double *__restrict__ dtau,
                          double *__restrict__ D, double *__restrict__ S,
                          double *__restrict__ gscratch) {
    const int f = blockIdx.x;
    if (f >= nfil) return;
    spline_quintic_fil(off[f], off[f + 1] - off[f], x, xn, dtau, D, S, gscratch);
}

// --------------------------------------------------------- segment geometry
struct GLArgs {
    double h[kMaxQ];
    double w[kMaxQ];
};

// Quadrature points, vector charges and segment lengths of segment j (in u
// in [0,1], tau = tau_j + u h; ds/dtau = s'(u)/h).  ORDER 4 writes the node's
// second derivative (from its segment's start); ORDER 6 reads it (solved
// with the slopes).
template <int ORDER>
__device__ __forceinline__ void geometry_seg(int j, int jn, double g, int Q, const GLArgs &gl,
                                             const double *__restrict__ x,
                                             const double *__restrict__ xn,
                                             const double *__restrict__ dtau,
                                             const double *__restrict__ D,
                                             double *__restrict__ qpos, double *__restrict__ qchg,
                                             double *__restrict__ sdd, double *__restrict__ ell) {
    const double h = dtau[j];
    SegPoly<ORDER> sp;
    sp.load(x, xn, j, D, sdd, j, jn, h);
    if constexpr (ORDER == 4) {
#pragma unroll
        for (int q = 0; q < 3; q++) sdd[3 * j + q] = 2.0 * sp.c[2][q] / (h * h);
    }
    double len = 0.0;
    for (int i = 0; i < Q; i++) {
        double u = gl.h[i], p[3], der[3];
        sp.pos(u, p);
        sp.der(u, der);
#pragma unroll
        for (int q = 0; q < 3; q++) {
            der[q] /= h;
            qpos[3 * (j * Q + i) + q] = p[q];
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

// 3-point Gauss-Legendre rule on [0, 1]
__device__ constexpr double kG3h[3] = {0.11270166537925831148, 0.5, 0.88729833462074168852};
__device__ constexpr double kG3w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

// Local terms (eq:BS_local, eq:streamfunction_local) and long-range self
// corrections.  With eps < 1 the local segments are subdivided (Sec. 5.2):
// the Taylor expansion covers the fraction eps of each local segment next
// to the node (l-, l+ the arc lengths of those portions, 3-point rule), and
// the rest of each segment is integrated with the unsplit kernels by
// 3-point rules on panels graded towards the node, [eps, 2 eps],
// [2 eps, 4 eps], ..., ending at the segment's far node.
struct LocalArgs {
    int Q, mode;
    double sign, a, delta, alpha, eps;
};

// node i with neighbours ip (previous) and in (next) on its filament.
// Segment ip lies in the frame of node ip, where node i sits at xn[ip]
// (x[i] plus the period shift when i is the first node of an infinite
// filament); segment i lies in the frame of node i.
template <int ORDER>
__device__ void local_self_node(int i, int ip, int in, double g, const LocalArgs &la,
                                const double *__restrict__ x, const double *__restrict__ xn,
                                const double *__restrict__ dtau,
                                const double *__restrict__ D, const double *__restrict__ sdd,
                                const double *__restrict__ ell, const double *__restrict__ qpos,
                                const double *__restrict__ qchg, double *__restrict__ out) {
    const int Q = la.Q, mode = la.mode;
    const double a = la.a, delta = la.delta, alpha = la.alpha, eps = la.eps, sign = la.sign;
    const double inv4pi = 1.0 / (4.0 * kPi);
    bool psi = (mode & LS_PSI) != 0;
    double acc[3] = {0.0, 0.0, 0.0};
    if (mode & LS_VLOCAL) {
        double sd[3] = {D[3 * i], D[3 * i + 1], D[3 * i + 2]};
        double sn = sqrt(sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]);
        double lm = ell[ip], lp = ell[i];
        const bool sub = eps < 1.0;
        SegPoly<ORDER> seg[2];
        if (sub) {
            seg[0].load(x, xn, ip, D, sdd, ip, i, dtau[ip]);
            seg[1].load(x, xn, i, D, sdd, i, in, dtau[i]);
            lm = lp = 0.0;
            for (int k = 0; k < 3; k++) {
                double dv[3];
                seg[0].der(1.0 - eps + kG3h[k] * eps, dv);
                lm += kG3w[k] * eps * sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                seg[1].der(kG3h[k] * eps, dv);
                lp += kG3w[k] * eps * sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            }
        }
        double lg = log(2.0 * sqrt(lm * lp) / a);
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
        if (sub) {
            // the rest of each local segment, distance u from the node in [eps, 1]
            for (int side = 0; side < 2; side++) {
                const double *xi = side ? x + 3 * i : xn + 3 * ip;
                for (double u0 = eps; u0 < 1.0; u0 *= 2.0) {
                    const double u1 = fmin(2.0 * u0, 1.0);
                    for (int k = 0; k < 3; k++) {
                        const double uu = u0 + kG3h[k] * (u1 - u0);
                        const double u = side ? uu : 1.0 - uu;
                        double p[3], dv[3], r[3];
                        seg[side].pos(u, p);
                        seg[side].der(u, dv);   // ds/du: ds = dv du
                        for (int q = 0; q < 3; q++) r[q] = p[q] - xi[q];
                        const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                        const double w = g * kG3w[k] * (u1 - u0) * inv4pi;
                        if (!psi) {
                            const double f = w / (rr * rr * rr);
                            acc[0] += f * (r[1] * dv[2] - r[2] * dv[1]);
                            acc[1] += f * (r[2] * dv[0] - r[0] * dv[2]);
                            acc[2] += f * (r[0] * dv[1] - r[1] * dv[0]);
                        } else {
                            const double f = w / rr;
                            for (int q = 0; q < 3; q++) acc[q] += f * dv[q];
                        }
                    }
                }
            }
        }
    }
    if (mode & LS_VSELF) {
        double self[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; s++)
            for (int k = 0; k < Q; k++) {
                const int qi = (s == 0 ? ip : i) * Q + k;
                const double *xi = s == 0 ? xn + 3 * ip : x + 3 * i;
                double r[3], c[3];
                for (int q = 0; q < 3; q++) r[q] = qpos[3 * qi + q] - xi[q];
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

template <int ORDER>
__global__ __launch_bounds__(256) void k_local_self(int N, LocalArgs la, const double *__restrict__ x,
                             const double *__restrict__ xn, const int *__restrict__ off, const int *__restrict__ fil,
                             const double *__restrict__ gamma, const double *__restrict__ dtau,
                             const double *__restrict__ D, const double *__restrict__ sdd,
                             const double *__restrict__ ell, const double *__restrict__ qpos,
                             const double *__restrict__ qchg, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    local_self_node<ORDER>(i, prev_node(off, fil, i), next_node(off, fil, i), gamma[fil[i]], la,
                           x, xn, dtau, D, sdd, ell, qpos, qchg, out);
}

// ----------------------------------------------------- one filament at once
// Everything set_filaments derives per filament, in one workgroup per
// filament: chord lengths (and the plan's copies of the nodes and of the
// circulation), the spline solve, quadrature points, charges and segment
// lengths, and (LOCAL) the velocity's local term minus the long-range self
// correction (into vls, which the velocity sums start from).  The keys and
// counts of the bin sorts that follow are formed here too.  The local term
// is what sets the kernel's registers (237 VGPRs with it, two wavefronts per
// SIMD; 82 without, five), so inputs that need more wavefronts than that
// leave it to k_local_self, one thread per node (1e6 nodes in 1e4 filaments:
// 0.40 -> 0.29 ms for both launches); the others keep the single launch.
template <int ORDER, bool LOCAL>
__global__ __launch_bounds__(128) void k_filament(int nfil, const int *__restrict__ off, const double *xs,
                           double *xd, double *__restrict__ xn,
                           const double *__restrict__ shift,
                           const double *__restrict__ gs, double *__restrict__ gd,
                           double *__restrict__ dtau, double *__restrict__ D,
                           double *__restrict__ sdd, double *__restrict__ qpos,
                           double *__restrict__ qchg, double *__restrict__ ell,
                           int *__restrict__ status, double *__restrict__ gscratch, GLArgs gl,
                           LocalArgs la, double *__restrict__ vls, BinKeys bk) {
    const int f = blockIdx.x;
    if (f >= nfil) return;
    const int b0 = off[f], n = off[f + 1] - off[f];
    chord_fil(f, b0, n, xs, xd, xn, shift, gs, gd, dtau, status);
    __syncthreads();
    if constexpr (ORDER == 4) spline_cubic_fil(b0, n, xd, xn, dtau, D, gscratch);
    else spline_quintic_fil(b0, n, xd, xn, dtau, D, sdd, gscratch);
    __syncthreads();
    const double g = gs[f];
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        geometry_seg<ORDER>(b0 + k, b0 + (k + 1 == n ? 0 : k + 1), g, la.Q, gl, xd, xn, dtau, D,
                            qpos, qchg, sdd, ell);
    __syncthreads();
    // bin keys and counts of the filament's quadrature points (spread tile,
    // pair cell) and nodes (pair cell); whole-workgroup trip counts, as the
    // counting is wavefront-aggregated
    const int nq = n * la.Q;
    for (int t0 = 0; t0 < nq; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        const bool act = t < nq;
        const int qi = b0 * la.Q + t;
        int k0 = 0, k1 = 0;
        if (act) {
            k0 = tile_key(qpos + 3 * qi, bk.L, bk.inv_h, bk.w, bk.n, bk.T, bk.NT);
            k1 = cell_key(qpos + 3 * qi, bk.L, bk.nc);
            bk.key[0][qi] = k0;
            bk.key[1][qi] = k1;
        }
        wave_add<false>(bk.cnt[0], k0, act);
        wave_add<false>(bk.cnt[1], k1, act);
    }
    for (int t0 = 0; t0 < n; t0 += blockDim.x) {
        const int t = t0 + threadIdx.x;
        const bool act = t < n;
        int k2 = 0;
        if (act) {
            k2 = cell_key(xd + 3 * (b0 + t), bk.L, bk.nc);
            bk.key[2][b0 + t] = k2;
        }
        wave_add<false>(bk.cnt[2], k2, act);
    }
    if constexpr (LOCAL) {
        for (int k = threadIdx.x; k < n; k += blockDim.x)
            local_self_node<ORDER>(b0 + k, b0 + (k == 0 ? n - 1 : k - 1),
                                   b0 + (k + 1 == n ? 0 : k + 1), g, la, xd, xn, dtau, D, sdd,
                                   ell, qpos, qchg, vls);
    }
}

// ------------------------------------------------------------------ launch
static inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

static LocalArgs local_args(bs_plan_t p, int mode, double sign) {
    LocalArgs la;
    la.Q = p->Q;
    la.mode = mode;
    la.sign = sign;
    la.a = p->prm.a;
    la.delta = p->prm.delta;
    la.alpha = p->prm.alpha;
    la.eps = p->prm.local_frac > 0.0 ? p->prm.local_frac : 1.0;
    return la;
}

// The local term takes its own launch on inputs of at least this many nodes
// when the per-filament kernel is short of wavefronts: more filaments than
// its registers let run at once (two wavefronts per SIMD: 1024 filaments of
// two wavefronts), or filaments so long (over 1024 nodes on average) that
// their workgroups loop over many nodes each.  Otherwise the extra launch
// costs more than it saves (1e5 nodes in 1000 filaments: 44 -> 51 us).
constexpr int64_t kFilamentSplitNodes = 16384;
constexpr int64_t kFilamentSplitFils = 1024;

void launch_filaments(bs_plan_t p, const double *xyz, const double *gamma) {
    if (p->N == 0) return;
    GLRule r = gl_rule(p->Q);
    GLArgs g;
    for (int i = 0; i < kMaxQ; i++) { g.h[i] = r.h[i]; g.w[i] = r.w[i]; }
    const LocalArgs la = local_args(p, LS_VLOCAL | LS_VSELF | LS_ASSIGN, 1.0);
    const bool split = p->N >= kFilamentSplitNodes &&
                       (p->nfil > kFilamentSplitFils || p->N > kFilamentSplitFils * p->nfil);
    auto kern = p->order == 6 ? (split ? k_filament<6, false> : k_filament<6, true>)
                              : (split ? k_filament<4, false> : k_filament<4, true>);
    hipLaunchKernelGGL(kern, dim3((unsigned)p->nfil), dim3(p->order == 6 ? 64 : 128), 0,
                       p->stream, (int)p->nfil, (const int *)p->d_off.p, xyz,
                       (double *)p->d_x.p, (double *)p->d_xn.p,
                       p->nper ? (const double *)p->d_shift.p : nullptr, gamma,
                       (double *)p->d_gamma.p,
                       (double *)p->d_dtau.p, (double *)p->d_D.p, (double *)p->d_sdd.p,
                       (double *)p->d_qpos.p, (double *)p->d_qchg.p, (double *)p->d_ell.p,
                       (int *)p->d_status.p, (double *)p->spline_tmp.p, g, la,
                       (double *)p->d_vls.p, bin_keys(p));
    if (split) launch_local_self(p, LS_VLOCAL | LS_VSELF | LS_ASSIGN, 1.0, (double *)p->d_vls.p);
}

void launch_spline_data(bs_plan_t p, const double *data, double *Dout, double *Sout) {
    if (p->order == 6)
        hipLaunchKernelGGL(k_spline5, dim3((unsigned)p->nfil), dim3(64), 0, p->stream,
                           (int)p->nfil, (const int *)p->d_off.p, data, (const double *)nullptr,
                           (const double *)p->d_dtau.p, Dout, Sout, (double *)p->spline_tmp.p);
    else
        hipLaunchKernelGGL(k_spline, dim3((unsigned)p->nfil), dim3(128), 0, p->stream,
                           (int)p->nfil, (const int *)p->d_off.p, data, (const double *)nullptr,
                           (const double *)p->d_dtau.p, Dout, (double *)p->spline_tmp.p);
}

void launch_local_self(bs_plan_t p, int mode, double sign, double *out) {
    auto kern = p->order == 6 ? k_local_self<6> : k_local_self<4>;
    hipLaunchKernelGGL(kern, dim3(blocks_for(p->N, 256)), dim3(256), 0, p->stream, (int)p->N,
                       local_args(p, mode, sign), (const double *)p->d_x.p,
                       (const double *)p->d_xn.p, (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_gamma.p, (const double *)p->d_dtau.p,
                       (const double *)p->d_D.p, (const double *)p->d_sdd.p,
                       (const double *)p->d_ell.p, (const double *)p->d_qpos.p,
                       (const double *)p->d_qchg.p, out);
}

}  // namespace bs
