// Near-singular correction (not in the paper; the paper notes that the
// Q-point rule degrades for close segments and subdivides only the local
// ones, Sec. 5.2).  For every node i and every segment j that is not one of
// the two segments adjacent to i and whose chord passes closer to s_i than
// ns_eta * ell_j, the Q-point sum of segment j is replaced by the integral of
// the full Biot-Savart kernel over the spline segment:
//   dv_i += (Gamma_j/4pi) int_seg (s - s_i) x ds / |s - s_i|^3  -  sum_Q(...)
// (the same image of the segment as the chord test, minimum image).
//
// Passes (all deterministic, no host synchronisation):
//   flag   one thread per node scans the quadrature points of the cells around
//          it (the pair cell list), tests each segment's chord once (at the
//          first of its quadrature points that lies in the scanned window),
//          and counts (pass 0) or writes (pass 1) the flagged pairs in scan
//          order into a per-node slice of the pair list;
//   integrate  one thread per pair: closest point of the cubic segment to the
//          target by Newton steps, then Gauss-Legendre panels graded
//          geometrically (ratio 3) away from it, 16 points per panel, float64;
//   apply  one thread per node adds its pairs' corrections in list order.
#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

constexpr int kNsGL = 16;
struct NsRule {
    double x[kNsGL];   // nodes on [-1, 1]
    double w[kNsGL];
};

// ------------------------------------------------------------ max segment
__global__ void k_max_ell(int N, const double *__restrict__ ell, double *__restrict__ out) {
    __shared__ double sh[256];
    double m = 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) m = fmax(m, ell[j]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__device__ __forceinline__ int cell_of(double v, double L, int nc) {
    int c = (int)(wrap_box(v, L) / L * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ bool in_window(int c, int c0, int span, int nc) {
    int d = c - c0;
    if (d < 0) d = -d;
    if (nc - d < d) d = nc - d;
    return d <= span;
}

// chord distance from x to segment A->B with A, B shifted by the minimum
// image of the chord midpoint; returns distance and the image shift of x
__device__ __forceinline__ double chord_dist(const double *A, const double *B, const double *x,
                                             double L, double *xs) {
    double e[3], r[3];
    for (int q = 0; q < 3; q++) {
        double m = 0.5 * (A[q] + B[q]);
        xs[q] = x[q] - L * rint((x[q] - m) / L);
        e[q] = B[q] - A[q];
        r[q] = xs[q] - A[q];
    }
    double ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    double t = (r[0] * e[0] + r[1] * e[1] + r[2] * e[2]) / ee;
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    double d0 = r[0] - t * e[0], d1 = r[1] - t * e[1], d2 = r[2] - t * e[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

struct NsArgs {
    int N, Q, nc, max_per_node;
    double L, eta;
    const double *x, *ell, *qpos, *maxell;
    const int *off, *fil, *nperm, *cstart, *sseg;
    const double4 *spos;
};

// One wavefront per node: lanes take consecutive quadrature points of each
// scanned cell; flagged lanes are ranked with a ballot so that pass 0 counts
// and pass 1 writes the pairs in scan order (cell order, then sorted order).
// pass 0: cnt[o] = number of flagged pairs; pass 1: write pairs at pstart[o]
template <int PASS>
__global__ __launch_bounds__(256) void k_ns_flag(NsArgs a, int *__restrict__ cnt,
                                                 const int *__restrict__ pstart,
                                                 int2 *__restrict__ pairs,
                                                 int *__restrict__ status) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gid >> 6, lane = gid & 63;
    if (t >= a.N) return;   // whole wavefronts exit together
    const int o = a.nperm[t];
    const int ip = prev_node_d(a.off, a.fil, o);
    const double xi[3] = {a.x[3 * o], a.x[3 * o + 1], a.x[3 * o + 2]};
    const int nc = a.nc;
    int c0[3];
    for (int q = 0; q < 3; q++) c0[q] = cell_of(xi[q], a.L, nc);
    const double cell = a.L / nc;
    int span = (int)ceil((a.eta + 1.25) * (*a.maxell) / cell);
    bool full = (2 * span + 1 >= nc);
    if (full) span = nc;   // every cell, once
    const int lo = full ? 0 : -span, hi = full ? nc - 1 : span;
    int k = 0;
    const int base = PASS ? pstart[o] : 0;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int dz = lo; dz <= hi; dz++) {
        int cz = full ? dz : c0[2] + dz;
        cz = cz < 0 ? cz + nc : (cz >= nc ? cz - nc : cz);
        for (int dy = lo; dy <= hi; dy++) {
            int cy = full ? dy : c0[1] + dy;
            cy = cy < 0 ? cy + nc : (cy >= nc ? cy - nc : cy);
            for (int dx = lo; dx <= hi; dx++) {
                int cx = full ? dx : c0[0] + dx;
                cx = cx < 0 ? cx + nc : (cx >= nc ? cx - nc : cx);
                const int cidx = (cz * nc + cy) * nc + cx;
                const int s = a.cstart[cidx], e = a.cstart[cidx + 1];
                for (int p0 = s; p0 < e; p0 += 64) {
                    const int p = p0 + lane;
                    bool flag = false;
                    int sg = -1;
                    double xs[3] = {0.0, 0.0, 0.0};
                    if (p < e) {
                        sg = a.sseg[p];
                        if (sg != o && sg != ip) {
                            int jn = next_node_d(a.off, a.fil, sg);
                            const double A[3] = {a.x[3 * sg], a.x[3 * sg + 1], a.x[3 * sg + 2]};
                            const double Bv[3] = {a.x[3 * jn], a.x[3 * jn + 1], a.x[3 * jn + 2]};
                            double d = chord_dist(A, Bv, xi, a.L, xs);
                            if (d < a.eta * a.ell[sg]) {
                                // count the segment once: at the first of its
                                // quadrature points inside the scanned window
                                double4 sp = a.spos[p];
                                int first = 0;
                                for (int i2 = 0; i2 < a.Q; i2++) {
                                    const double *qp = a.qpos + 3 * ((size_t)sg * a.Q + i2);
                                    bool inw = full ||
                                               (in_window(cell_of(qp[0], a.L, nc), c0[0], span, nc) &&
                                                in_window(cell_of(qp[1], a.L, nc), c0[1], span, nc) &&
                                                in_window(cell_of(qp[2], a.L, nc), c0[2], span, nc));
                                    if (inw) { first = i2; break; }
                                }
                                const double *qf = a.qpos + 3 * ((size_t)sg * a.Q + first);
                                flag = wrap_box(qf[0], a.L) == sp.x && wrap_box(qf[1], a.L) == sp.y &&
                                       wrap_box(qf[2], a.L) == sp.z;
                            }
                        }
                    }
                    const unsigned long long m = __ballot(flag);
                    if (PASS && flag) {
                        int slot = k + __popcll(m & below);
                        if (slot < a.max_per_node) {
                            // image shift of the target, periods per axis,
                            // packed as three 10-bit fields (+-511 periods)
                            int sh = 0;
                            for (int q = 0; q < 3; q++) {
                                int sv = (int)rint((xs[q] - xi[q]) / a.L);
                                sv = sv < -511 ? -511 : (sv > 511 ? 511 : sv);
                                sh = (sh << 10) | (sv + 512);
                            }
                            pairs[base + slot] = make_int2(sg, sh);
                        }
                    }
                    k += __popcll(m);
                }
            }
        }
    }
    if (PASS == 0 && lane == 0) {
        if (k > a.max_per_node) atomicOr(status, 2);
        cnt[o] = k < a.max_per_node ? k : a.max_per_node;
    }
}

// cubic Hermite segment j as c0 + c1 u + c2 u^2 + c3 u^3
struct Seg {
    double c0[3], c1[3], c2[3], c3[3];
};

__device__ __forceinline__ Seg load_seg(int j, const int *off, const int *fil, const double *x,
                                        const double *D, const double *dtau) {
    Seg s;
    int jn = next_node_d(off, fil, j);
    double h = dtau[j];
    for (int q = 0; q < 3; q++) {
        double s0 = x[3 * j + q], s1 = x[3 * jn + q];
        double d0 = h * D[3 * j + q], d1 = h * D[3 * jn + q];
        s.c0[q] = s0;
        s.c1[q] = d0;
        s.c2[q] = 3.0 * (s1 - s0) - 2.0 * d0 - d1;
        s.c3[q] = 2.0 * (s0 - s1) + d0 + d1;
    }
    return s;
}

// integral over u in [a, b] of (s(u) - x) x s'(u) / |s(u) - x|^3 with
// kNsGL-point Gauss-Legendre
__device__ void ns_panel(const Seg &s, const double *x, double a, double b, const NsRule &R,
                         double *acc) {
    double m = 0.5 * (a + b), hw = 0.5 * (b - a);
    for (int k = 0; k < kNsGL; k++) {
        double u = m + hw * R.x[k];
        double r[3], d[3];
        for (int q = 0; q < 3; q++) {
            r[q] = s.c0[q] + u * (s.c1[q] + u * (s.c2[q] + u * s.c3[q])) - x[q];
            d[q] = s.c1[q] + u * (2.0 * s.c2[q] + 3.0 * u * s.c3[q]);
        }
        double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double f = R.w[k] * hw / (r2 * sqrt(r2));
        acc[0] += f * (r[1] * d[2] - r[2] * d[1]);
        acc[1] += f * (r[2] * d[0] - r[0] * d[2]);
        acc[2] += f * (r[0] * d[1] - r[1] * d[0]);
    }
}

// Integral over u in [0,1] of (s(u) - x) x s'(u) / |s(u) - x|^3 for one
// cubic segment: closest point by a coarse scan and Newton steps on
// (s - x) . s' = 0, then 16-point Gauss-Legendre panels graded geometrically
// (ratio 3) away from it.
__device__ __forceinline__ void seg_eval(const Seg &s, double u, double *p, double *d1) {
    for (int q = 0; q < 3; q++) {
        p[q] = s.c0[q] + u * (s.c1[q] + u * (s.c2[q] + u * s.c3[q]));
        d1[q] = s.c1[q] + u * (2.0 * s.c2[q] + 3.0 * u * s.c3[q]);
    }
}

// parameter of the point of the segment closest to x: best of a coarse scan,
// then Newton steps on (s - x) . s' = 0 kept inside [0, 1]
__device__ double closest_u(const Seg &s, const double *xs) {
    double ub = 0.0, best = 1e300;
    for (int k = 0; k <= 8; k++) {
        double u = k / 8.0, r2 = 0.0;
        for (int q = 0; q < 3; q++) {
            double r = s.c0[q] + u * (s.c1[q] + u * (s.c2[q] + u * s.c3[q])) - xs[q];
            r2 += r * r;
        }
        if (r2 < best) { best = r2; ub = u; }
    }
    for (int it = 0; it < 8; it++) {
        double g = 0.0, dg = 0.0;
        for (int q = 0; q < 3; q++) {
            double r = s.c0[q] + ub * (s.c1[q] + ub * (s.c2[q] + ub * s.c3[q])) - xs[q];
            double d1 = s.c1[q] + ub * (2.0 * s.c2[q] + 3.0 * ub * s.c3[q]);
            double d2 = 2.0 * s.c2[q] + 6.0 * ub * s.c3[q];
            g += r * d1;
            dg += d1 * d1 + r * d2;
        }
        if (!(dg > 0.0)) break;
        double un = ub - g / dg;
        un = un < 0.0 ? 0.0 : (un > 1.0 ? 1.0 : un);
        ub = un;
    }
    return ub;
}

__device__ void ns_seg_integral(const Seg &s, const double *xs, const NsRule &R, double *acc) {
    const double ub = closest_u(s, xs);
    double P[3], d1[3];
    seg_eval(s, ub, P, d1);
    const double r2 = (P[0] - xs[0]) * (P[0] - xs[0]) + (P[1] - xs[1]) * (P[1] - xs[1]) +
                      (P[2] - xs[2]) * (P[2] - xs[2]);
    const double sp2 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    // half the distance in parameter units: the first panel pair is finer
    // than the singularity's width
    double delta = 0.5 * sqrt(r2 / sp2);
    delta = delta < 1e-13 ? 1e-13 : delta;
    acc[0] = acc[1] = acc[2] = 0.0;
    double a0 = ub - delta < 0.0 ? 0.0 : ub - delta, b0 = ub + delta > 1.0 ? 1.0 : ub + delta;
    if (b0 > a0) ns_panel(s, xs, a0, b0, R, acc);
    double edge = a0, width = delta;
    while (edge > 0.0) {
        double nxt = ub - 3.0 * width;
        if (nxt < 0.0) nxt = 0.0;
        ns_panel(s, xs, nxt, edge, R, acc);
        edge = nxt;
        width *= 3.0;
    }
    edge = b0; width = delta;
    while (edge < 1.0) {
        double nxt = ub + 3.0 * width;
        if (nxt > 1.0) nxt = 1.0;
        ns_panel(s, xs, edge, nxt, R, acc);
        edge = nxt;
        width *= 3.0;
    }
}

// (s_q - x) x q / |s_q - x|^3 summed over the Q points of segment sg
__device__ void ns_qsum(int sg, const double *xs, const double *qpos, const double *qchg, int Q,
                        double *qs) {
    qs[0] = qs[1] = qs[2] = 0.0;
    for (int i = 0; i < Q; i++) {
        const double *qp = qpos + 3 * ((size_t)sg * Q + i), *qc = qchg + 3 * ((size_t)sg * Q + i);
        double r[3] = {qp[0] - xs[0], qp[1] - xs[1], qp[2] - xs[2]};
        double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double f = 1.0 / (rr2 * sqrt(rr2));
        qs[0] += f * (r[1] * qc[2] - r[2] * qc[1]);
        qs[1] += f * (r[2] * qc[0] - r[0] * qc[2]);
        qs[2] += f * (r[0] * qc[1] - r[1] * qc[0]);
    }
}

__device__ __forceinline__ void unpack_shift(int sh, const double *x, double L, double *xs) {
    int shv[3] = {((sh >> 20) & 1023) - 512, ((sh >> 10) & 1023) - 512, (sh & 1023) - 512};
    for (int q = 0; q < 3; q++) xs[q] = x[q] + shv[q] * L;
}

// Exact segment integral minus its Q-point sum, for one (node, segment) pair.
__device__ void ns_pair(int o, int sg, int sh, const int *off, const int *fil, const double *x,
                        const double *D, const double *dtau, const double *gamma,
                        const double *qpos, const double *qchg, int Q, double L,
                        const NsRule &R, double *out) {
    double xs[3];
    unpack_shift(sh, x + 3 * o, L, xs);
    Seg s = load_seg(sg, off, fil, x, D, dtau);
    double acc[3], qs[3];
    ns_seg_integral(s, xs, R, acc);
    ns_qsum(sg, xs, qpos, qchg, Q, qs);
    const double g4 = gamma[fil[sg]] / (4.0 * kPi);
    for (int q = 0; q < 3; q++) out[q] = g4 * acc[q] - qs[q] / (4.0 * kPi);
}

__global__ __launch_bounds__(256) void k_ns_integrate(
    const int *__restrict__ total, const int *__restrict__ pnode, const int2 *__restrict__ pairs,
    const int *__restrict__ off, const int *__restrict__ fil, const double *__restrict__ x,
    const double *__restrict__ D, const double *__restrict__ dtau,
    const double *__restrict__ gamma, const double *__restrict__ qpos,
    const double *__restrict__ qchg, int Q, double L, NsRule R, double *__restrict__ pout) {
    const int P = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        int2 pr = pairs[p];
        double out[3];
        ns_pair(pnode[p], pr.x, pr.y, off, fil, x, D, dtau, gamma, qpos, qchg, Q, L, R, out);
        pout[3 * (size_t)p] = out[0];
        pout[3 * (size_t)p + 1] = out[1];
        pout[3 * (size_t)p + 2] = out[2];
    }
}

// owner node of each pair slot (for the per-pair kernel)
__global__ void k_ns_owner(int N, const int *__restrict__ pstart, int *__restrict__ pnode) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    for (int p = pstart[o]; p < pstart[o + 1]; p++) pnode[p] = o;
}

__global__ void k_ns_apply(int N, const int *__restrict__ pstart, const double *__restrict__ pout,
                           double *__restrict__ v) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int p = pstart[o]; p < pstart[o + 1]; p++) {
        s0 += pout[3 * (size_t)p];
        s1 += pout[3 * (size_t)p + 1];
        s2 += pout[3 * (size_t)p + 2];
    }
    v[3 * o] += s0;
    v[3 * o + 1] += s1;
    v[3 * o + 2] += s2;
}

// ------------------------------------------------------ learned correction
// Chord frame of a segment A -> B (node slopes D0, D1): e1 along the chord,
// e2 along the part of D0 normal to it (else of D1, else any normal), e3 =
// e1 x e2; lengths in units of the chord h.  Features (8, float32):
//   (x - M).e_k / h (3),  D0.e1, D0.e2,  D1.e1, D1.e2, D1.e3
// with M the chord midpoint.  The segment in this frame is the cubic from
// (-1/2,0,0) to (1/2,0,0) with end derivatives D0, D1 (chord-length knots
// make d tau = h), so the integral is a function of the 8 features alone
// (times 1/h).  The network predicts z = (I_seg - I_tan) / |I_tan| in frame
// components, I_tan the integral over the straight segment tangent to the
// curve at its point closest to the target (distance d), which carries the
// 1/d singularity exactly: z is a relative remainder, so the squared loss is
// the mean squared relative error of the learned integral.
constexpr double kNsThetaMax = 0.6;     // max angle of D0, D1 to the chord
constexpr double kNsDmin = 0.9, kNsDmax = 1.1;   // |D0|, |D1| range
constexpr double kNsRlo = 1e-3, kNsRhi = 1.1;    // d_c / h range
constexpr int kNsBins = 12;                      // log10(d_c/h) bins of the error table

struct NsBox {
    float err[kNsBins];   // max relative error of the learned integral per bin
    double tol;           // fall back where err > tol
};

// raw straight-segment integral  int (s - x) x ds / |s - x|^3  over A -> B
__device__ __forceinline__ void chord_raw(const double *A, const double *B, const double *x,
                                          double *out) {
    double r1[3] = {A[0] - x[0], A[1] - x[1], A[2] - x[2]};
    double r2[3] = {B[0] - x[0], B[1] - x[1], B[2] - x[2]};
    double p = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    double q = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
    double c[3] = {r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2],
                   r1[0] * r2[1] - r1[1] * r2[0]};
    double dt = r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2];
    // p q + r1.r2 cancels when the target lies beside the segment; there it
    // equals |r1 x r2|^2 / (p q - r1.r2)
    double den = dt >= 0.0 ? p * q + dt : (c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) / (p * q - dt);
    double f = (p + q) / (p * q * den);
    out[0] = c[0] * f; out[1] = c[1] * f; out[2] = c[2] * f;
}

// Straight segment tangent to the curve at its point P closest to x, running
// |P - s(0)| back and |s(1) - P| forward along the unit tangent: it carries
// the same 1/d singularity as the curve (d = |P - x|), so the remainder
// I_seg - I_tan is small relative to I_tan near the curve.  Returns I_tan
// (raw integral), the scale |I_tan| the network's output is multiplied by,
// and d/h.
__device__ void tangent_baseline(const Seg &s, const double *x, double h, double *Itan,
                                 double *scale, double *dstar) {
    const double u = closest_u(s, x);
    double P[3], d1[3], S0[3], S1[3], dummy[3];
    seg_eval(s, u, P, d1);
    seg_eval(s, 0.0, S0, dummy);
    seg_eval(s, 1.0, S1, dummy);
    double tn = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
    double a = 0.0, b = 0.0, d = 0.0;
    for (int q = 0; q < 3; q++) {
        a += (P[q] - S0[q]) * (P[q] - S0[q]);
        b += (S1[q] - P[q]) * (S1[q] - P[q]);
        d += (P[q] - x[q]) * (P[q] - x[q]);
    }
    a = sqrt(a); b = sqrt(b); d = sqrt(d);
    double A[3], B[3];
    for (int q = 0; q < 3; q++) {
        A[q] = P[q] - a * d1[q] / tn;
        B[q] = P[q] + b * d1[q] / tn;
    }
    chord_raw(A, B, x, Itan);
    double m = sqrt(Itan[0] * Itan[0] + Itan[1] * Itan[1] + Itan[2] * Itan[2]);
    *scale = m > 1e-300 ? m : 1e-300;
    *dstar = d / h;
}

struct NsFrame {
    double e[3][3];
    double h, dc;   // chord length, distance to the chord over h
    float f[8];
    bool inbox;
};

__device__ NsFrame ns_frame(const double *A, const double *B, const double *D0, const double *D1,
                            const double *x) {
    NsFrame F;
    double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    F.h = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double *e1 = F.e[0], *e2 = F.e[1], *e3 = F.e[2];
    for (int q = 0; q < 3; q++) e1[q] = d[q] / F.h;
    double a0 = D0[0] * e1[0] + D0[1] * e1[1] + D0[2] * e1[2];
    double a1 = D1[0] * e1[0] + D1[1] * e1[1] + D1[2] * e1[2];
    double p0[3], p1[3];
    for (int q = 0; q < 3; q++) { p0[q] = D0[q] - a0 * e1[q]; p1[q] = D1[q] - a1 * e1[q]; }
    double n0 = sqrt(p0[0] * p0[0] + p0[1] * p0[1] + p0[2] * p0[2]);
    double n1 = sqrt(p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2]);
    if (n0 > 1e-12) for (int q = 0; q < 3; q++) e2[q] = p0[q] / n0;
    else if (n1 > 1e-12) for (int q = 0; q < 3; q++) e2[q] = p1[q] / n1;
    else {
        int k = (fabs(e1[0]) < fabs(e1[1])) ? (fabs(e1[0]) < fabs(e1[2]) ? 0 : 2)
                                            : (fabs(e1[1]) < fabs(e1[2]) ? 1 : 2);
        double u[3] = {0.0, 0.0, 0.0};
        u[k] = 1.0;
        double t = u[0] * e1[0] + u[1] * e1[1] + u[2] * e1[2];
        for (int q = 0; q < 3; q++) u[q] -= t * e1[q];
        double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int q = 0; q < 3; q++) e2[q] = u[q] / nu;
    }
    e3[0] = e1[1] * e2[2] - e1[2] * e2[1];
    e3[1] = e1[2] * e2[0] - e1[0] * e2[2];
    e3[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double xl[3];
    for (int k = 0; k < 3; k++) {
        double s = 0.0;
        for (int q = 0; q < 3; q++) s += (x[q] - 0.5 * (A[q] + B[q])) * F.e[k][q];
        xl[k] = s / F.h;
    }
    double b0 = D0[0] * e2[0] + D0[1] * e2[1] + D0[2] * e2[2];
    double b1 = D1[0] * e2[0] + D1[1] * e2[1] + D1[2] * e2[2];
    double c1 = D1[0] * e3[0] + D1[1] * e3[1] + D1[2] * e3[2];
    F.f[0] = (float)xl[0]; F.f[1] = (float)xl[1]; F.f[2] = (float)xl[2];
    F.f[3] = (float)a0; F.f[4] = (float)b0; F.f[5] = (float)a1; F.f[6] = (float)b1;
    F.f[7] = (float)c1;
    double tc = xl[0] + 0.5;
    double tcl = tc < 0.0 ? 0.0 : (tc > 1.0 ? 1.0 : tc);
    F.dc = sqrt((tc - tcl) * (tc - tcl) + xl[1] * xl[1] + xl[2] * xl[2]);
    double m0 = sqrt(a0 * a0 + b0 * b0), m1 = sqrt(a1 * a1 + b1 * b1 + c1 * c1);
    double th0 = atan2(b0, a0), th1 = atan2(sqrt(b1 * b1 + c1 * c1), a1);
    F.inbox = F.dc >= kNsRlo && F.dc <= kNsRhi && m0 >= kNsDmin && m0 <= kNsDmax &&
              m1 >= kNsDmin && m1 <= kNsDmax && th0 <= kNsThetaMax && th1 <= kNsThetaMax;
    return F;
}

__device__ __forceinline__ int ns_bin(double dc) {
    double t = (log10(dc) - log10(kNsRlo)) / (log10(kNsRhi) - log10(kNsRlo));
    int b = (int)(t * kNsBins);
    return b < 0 ? 0 : (b >= kNsBins ? kNsBins - 1 : b);
}

// Training samples from caller-supplied uniforms U[n][8]: tangent angles and
// lengths (U0..U4), position class and parameter (U5), distance (U6,
// log-uniform over [kNsRlo, kNsRhi]) and azimuth (U7).  70 % of targets lie
// beside the chord, 30 % on the hemispherical caps beyond either end.
__global__ void k_ns_samples(int64_t n, const double *__restrict__ U, NsRule R,
                             float *__restrict__ X, float *__restrict__ T,
                             double *__restrict__ aux) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *u = U + 8 * i;
    double th0 = kNsThetaMax * u[0], m0 = kNsDmin + (kNsDmax - kNsDmin) * u[1];
    double th1 = kNsThetaMax * u[2], ps1 = 2.0 * kPi * u[3], m1 = kNsDmin + (kNsDmax - kNsDmin) * u[4];
    double D0[3] = {m0 * cos(th0), m0 * sin(th0), 0.0};
    double D1[3] = {m1 * cos(th1), m1 * sin(th1) * cos(ps1), m1 * sin(th1) * sin(ps1)};
    double dc = kNsRlo * pow(kNsRhi / kNsRlo, u[6]), ph = 2.0 * kPi * u[7];
    double x[3];
    if (u[5] < 0.7) {
        double tc = u[5] / 0.7;
        x[0] = tc - 0.5; x[1] = dc * cos(ph); x[2] = dc * sin(ph);
    } else {
        double v = (u[5] - 0.7) / 0.3;
        double sg = v < 0.5 ? -1.0 : 1.0;
        double ct = 2.0 * v - floor(2.0 * v), st = sqrt(1.0 - ct * ct);
        x[0] = sg * (0.5 + dc * ct); x[1] = dc * st * cos(ph); x[2] = dc * st * sin(ph);
    }
    const double A[3] = {-0.5, 0.0, 0.0}, B[3] = {0.5, 0.0, 0.0};
    Seg s;
    for (int q = 0; q < 3; q++) {
        s.c0[q] = A[q];
        s.c1[q] = D0[q];
        s.c2[q] = 3.0 * (B[q] - A[q]) - 2.0 * D0[q] - D1[q];
        s.c3[q] = 2.0 * (A[q] - B[q]) + D0[q] + D1[q];
    }
    double I[3], It[3], scale, dstar;
    ns_seg_integral(s, x, R, I);
    tangent_baseline(s, x, 1.0, It, &scale, &dstar);
    NsFrame F = ns_frame(A, B, D0, D1, x);
    for (int k = 0; k < 8; k++) X[8 * i + k] = F.f[k];
    for (int q = 0; q < 3; q++) T[3 * i + q] = (float)((I[q] - It[q]) / scale);
    if (aux) {
        aux[6 * i] = dstar;
        aux[6 * i + 1] = I[0]; aux[6 * i + 2] = I[1]; aux[6 * i + 3] = I[2];
        aux[6 * i + 4] = scale;
        aux[6 * i + 5] = F.dc;
    }
}

__device__ __forceinline__ void pair_geometry(int o, int sg, int sh, const int *off, const int *fil,
                                              const double *x, const double *D, double L,
                                              double *A, double *B, double *D0, double *D1,
                                              double *xs) {
    int jn = next_node_d(off, fil, sg);
    for (int q = 0; q < 3; q++) {
        A[q] = x[3 * sg + q]; B[q] = x[3 * jn + q];
        D0[q] = D[3 * sg + q]; D1[q] = D[3 * jn + q];
    }
    unpack_shift(sh, x + 3 * o, L, xs);
}

__global__ __launch_bounds__(256) void k_ns_features(
    const int *__restrict__ total, const int *__restrict__ pnode, const int2 *__restrict__ pairs,
    const int *__restrict__ off, const int *__restrict__ fil, const double *__restrict__ x,
    const double *__restrict__ D, double L, float *__restrict__ X) {
    const int P = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        int2 pr = pairs[p];
        double A[3], B[3], D0[3], D1[3], xs[3];
        pair_geometry(pnode[p], pr.x, pr.y, off, fil, x, D, L, A, B, D0, D1, xs);
        NsFrame F = ns_frame(A, B, D0, D1, xs);
        for (int k = 0; k < 8; k++) X[8 * (size_t)p + k] = F.f[k];
    }
}

// learned integral where the error table allows it, adaptive elsewhere
__global__ __launch_bounds__(256) void k_ns_combine(
    const int *__restrict__ total, const int *__restrict__ pnode, const int2 *__restrict__ pairs,
    const int *__restrict__ off, const int *__restrict__ fil, const double *__restrict__ x,
    const double *__restrict__ D, const double *__restrict__ dtau,
    const double *__restrict__ gamma, const double *__restrict__ qpos,
    const double *__restrict__ qchg, int Q, double L, NsRule R, NsBox box,
    const float *__restrict__ Y, double *__restrict__ pout, int *__restrict__ nfallback) {
    const int P = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        int2 pr = pairs[p];
        const int o = pnode[p];
        double A[3], B[3], D0[3], D1[3], xs[3];
        pair_geometry(o, pr.x, pr.y, off, fil, x, D, L, A, B, D0, D1, xs);
        NsFrame F = ns_frame(A, B, D0, D1, xs);
        Seg sgm = load_seg(pr.x, off, fil, x, D, dtau);
        double It[3], scale, dstar;
        tangent_baseline(sgm, xs, F.h, It, &scale, &dstar);
        double out[3];
        if (!F.inbox || (double)box.err[ns_bin(dstar)] > box.tol) {
            ns_pair(o, pr.x, pr.y, off, fil, x, D, dtau, gamma, qpos, qchg, Q, L, R, out);
            atomicAdd(nfallback, 1);
        } else {
            double qs[3], y[3];
            for (int k = 0; k < 3; k++) y[k] = (double)Y[3 * (size_t)p + k] * scale;
            ns_qsum(pr.x, xs, qpos, qchg, Q, qs);
            const double g4 = gamma[fil[pr.x]] / (4.0 * kPi);
            for (int q = 0; q < 3; q++) {
                double yw = F.e[0][q] * y[0] + F.e[1][q] * y[1] + F.e[2][q] * y[2];
                out[q] = g4 * (It[q] + yw / F.h) - qs[q] / (4.0 * kPi);
            }
        }
        pout[3 * (size_t)p] = out[0];
        pout[3 * (size_t)p + 1] = out[1];
        pout[3 * (size_t)p + 2] = out[2];
    }
}

static NsArgs ns_args(bs_plan_t p) {
    NsArgs a;
    a.N = (int)p->N; a.Q = p->Q; a.nc = p->nc; a.max_per_node = p->ns_max_per_node;
    a.L = p->prm.L; a.eta = p->prm.ns_eta;
    a.x = (const double *)p->d_x.p; a.ell = (const double *)p->d_ell.p;
    a.qpos = (const double *)p->d_qpos.p; a.maxell = (const double *)p->ns_maxell.p;
    a.off = (const int *)p->d_off.p; a.fil = (const int *)p->d_fil.p;
    a.nperm = (const int *)p->nd_perm.p; a.cstart = (const int *)p->pq_start.p;
    a.sseg = (const int *)p->pq_seg.p; a.spos = (const double4 *)p->pq_pos.p;
    return a;
}

// flag + list build (after geometry and binning)
void ns_build_pairs(bs_plan_t p) {
    const int N = (int)p->N;
    dim3 grid(ceil_div(N, 256)), block(256);
    dim3 wgrid(ceil_div((int64_t)N * 64, 256));
    hipLaunchKernelGGL(k_max_ell, dim3(1), dim3(256), 0, p->stream, N,
                       (const double *)p->d_ell.p, (double *)p->ns_maxell.p);
    NsArgs a = ns_args(p);
    int *cnt = (int *)p->ns_cnt.p, *start = (int *)p->ns_start.p;
    hipLaunchKernelGGL((k_ns_flag<0>), wgrid, block, 0, p->stream, a, cnt, (const int *)nullptr,
                       (int2 *)nullptr, (int *)p->d_status.p);
    exclusive_scan(p, cnt, start, N);
    hipLaunchKernelGGL((k_ns_flag<1>), wgrid, block, 0, p->stream, a, (int *)nullptr, start,
                       (int2 *)p->ns_pairs.p, (int *)p->d_status.p);
    hipLaunchKernelGGL(k_ns_owner, grid, block, 0, p->stream, N, start, (int *)p->ns_pnode.p);
}

void ns_rule(NsRule *R);

void launch_ns_adaptive(bs_plan_t p, double *v) {
    const int N = (int)p->N;
    NsRule R;
    ns_rule(&R);
    const int *start = (const int *)p->ns_start.p;
    hipLaunchKernelGGL(k_ns_integrate, dim3(1024), dim3(256), 0, p->stream, start + N,
                       (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_D.p,
                       (const double *)p->d_dtau.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_qpos.p, (const double *)p->d_qchg.p, p->Q,
                       p->prm.L, R, (double *)p->ns_pout.p);
    hipLaunchKernelGGL(k_ns_apply, dim3(ceil_div(N, 256)), dim3(256), 0, p->stream, N, start,
                       (const double *)p->ns_pout.p, v);
}

void launch_ns_mlp(bs_plan_t p, double *v) {
    const int N = (int)p->N;
    NsRule R;
    ns_rule(&R);
    const int *start = (const int *)p->ns_start.p;
    const int *total = start + N;
    hipLaunchKernelGGL(k_ns_features, dim3(1024), dim3(256), 0, p->stream, total,
                       (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_D.p, p->prm.L,
                       (float *)p->ns_X.p);
    mlp_forward_device(p->mlp, total, (int64_t)N * p->ns_max_per_node, (const float *)p->ns_X.p,
                       (float *)p->ns_Y.p, p->stream);
    NsBox box;
    for (int b = 0; b < kNsBins; b++) box.err[b] = p->ns_err[b];
    box.tol = p->prm.tol;
    hipLaunchKernelGGL(k_ns_combine, dim3(1024), dim3(256), 0, p->stream, total,
                       (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_D.p,
                       (const double *)p->d_dtau.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_qpos.p, (const double *)p->d_qchg.p, p->Q,
                       p->prm.L, R, box, (const float *)p->ns_Y.p, (double *)p->ns_pout.p,
                       (int *)p->ns_fallback.p);
    hipLaunchKernelGGL(k_ns_apply, dim3(ceil_div(N, 256)), dim3(256), 0, p->stream, N, start,
                       (const double *)p->ns_pout.p, v);
}

}  // namespace bs

extern "C" int bs_ns_samples(int64_t n, const double *U, float *X, float *T, double *aux,
                             void *hip_stream) {
    if (n < 0 || (n > 0 && (!U || !X || !T))) return BS_EINVAL;
    if (n == 0) return BS_OK;
    bs::NsRule R;
    bs::ns_rule(&R);
    hipLaunchKernelGGL(bs::k_ns_samples, dim3((unsigned)((n + 127) / 128)), dim3(128), 0,
                       (hipStream_t)hip_stream, n, U, R, X, T, aux);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

extern "C" int bs_ns_error_bins(double *lo, double *hi, int *nbins) {
    if (lo) *lo = bs::kNsRlo;
    if (hi) *hi = bs::kNsRhi;
    if (nbins) *nbins = bs::kNsBins;
    return BS_OK;
}
