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

// pass 0: cnt[o] = number of flagged pairs; pass 1: write pairs at pstart[o]
template <int PASS>
__global__ __launch_bounds__(256) void k_ns_flag(NsArgs a, int *__restrict__ cnt,
                                                 const int *__restrict__ pstart,
                                                 int2 *__restrict__ pairs,
                                                 int *__restrict__ status) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.N) return;
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
    int k = 0, base = PASS ? pstart[o] : 0;
    for (int dz = lo; dz <= hi; dz++) {
        int cz = full ? dz : c0[2] + dz;
        cz = cz < 0 ? cz + nc : (cz >= nc ? cz - nc : cz);
        for (int dy = lo; dy <= hi; dy++) {
            int cy = full ? dy : c0[1] + dy;
            cy = cy < 0 ? cy + nc : (cy >= nc ? cy - nc : cy);
            for (int dx = lo; dx <= hi; dx++) {
                int cx = full ? dx : c0[0] + dx;
                cx = cx < 0 ? cx + nc : (cx >= nc ? cx - nc : cx);
                int cidx = (cz * nc + cy) * nc + cx;
                for (int p = a.cstart[cidx]; p < a.cstart[cidx + 1]; p++) {
                    int sg = a.sseg[p];
                    if (sg == o || sg == ip) continue;
                    // quadrature index of this point within its segment: the
                    // sorted copy keeps the original index order inside a cell,
                    // so recover it from the position match
                    int jn = next_node_d(a.off, a.fil, sg);
                    const double A[3] = {a.x[3 * sg], a.x[3 * sg + 1], a.x[3 * sg + 2]};
                    const double Bv[3] = {a.x[3 * jn], a.x[3 * jn + 1], a.x[3 * jn + 2]};
                    double xs[3];
                    double d = chord_dist(A, Bv, xi, a.L, xs);
                    if (!(d < a.eta * a.ell[sg])) continue;
                    // canonical point: the first quadrature point of segment sg
                    // inside the scanned window
                    double4 sp = a.spos[p];
                    int first = -1;
                    for (int i2 = 0; i2 < a.Q; i2++) {
                        const double *qp = a.qpos + 3 * ((size_t)sg * a.Q + i2);
                        int qc[3] = {cell_of(qp[0], a.L, nc), cell_of(qp[1], a.L, nc),
                                     cell_of(qp[2], a.L, nc)};
                        bool inw = full || (in_window(qc[0], c0[0], span, nc) &&
                                            in_window(qc[1], c0[1], span, nc) &&
                                            in_window(qc[2], c0[2], span, nc));
                        if (inw) { first = i2; break; }
                    }
                    // is this point that first one?  compare wrapped positions
                    const double *qf = a.qpos + 3 * ((size_t)sg * a.Q + (first < 0 ? 0 : first));
                    bool same = wrap_box(qf[0], a.L) == sp.x && wrap_box(qf[1], a.L) == sp.y &&
                                wrap_box(qf[2], a.L) == sp.z;
                    if (!same) continue;
                    if (k < a.max_per_node) {
                        if (PASS) {
                            // image shift of the target, periods per axis,
                            // packed as three 10-bit fields (+-511 periods)
                            int sh = 0;
                            for (int q = 0; q < 3; q++) {
                                int s = (int)rint((xs[q] - xi[q]) / a.L);
                                s = s < -511 ? -511 : (s > 511 ? 511 : s);
                                sh = (sh << 10) | (s + 512);
                            }
                            pairs[base + k] = make_int2(sg, sh);
                        }
                    } else if (PASS == 0) {
                        atomicOr(status, 2);
                    }
                    k++;
                }
            }
        }
    }
    if (PASS == 0) cnt[o] = k < a.max_per_node ? k : a.max_per_node;
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

// Exact segment integral minus its Q-point sum, for one (node, segment) pair.
__device__ void ns_pair(int o, int sg, int sh, const int *off, const int *fil, const double *x,
                        const double *D, const double *dtau, const double *gamma,
                        const double *qpos, const double *qchg, int Q, double L,
                        const NsRule &R, double *out) {
    double xs[3];
    int shv[3] = {((sh >> 20) & 1023) - 512, ((sh >> 10) & 1023) - 512, (sh & 1023) - 512};
    for (int q = 0; q < 3; q++) xs[q] = x[3 * o + q] + shv[q] * L;
    Seg s = load_seg(sg, off, fil, x, D, dtau);
    // closest point: best of a coarse scan, then Newton on (s - x) . s' = 0
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
    double r2 = 0.0, sp2 = 0.0;
    for (int q = 0; q < 3; q++) {
        double r = s.c0[q] + ub * (s.c1[q] + ub * (s.c2[q] + ub * s.c3[q])) - xs[q];
        double d1 = s.c1[q] + ub * (2.0 * s.c2[q] + 3.0 * ub * s.c3[q]);
        r2 += r * r;
        sp2 += d1 * d1;
    }
    // half the distance in parameter units: the first panel pair is finer
    // than the singularity's width
    double delta = 0.5 * sqrt(r2 / sp2);
    delta = delta < 1e-13 ? 1e-13 : delta;
    double acc[3] = {0.0, 0.0, 0.0};
    // centre panel
    double a0 = ub - delta < 0.0 ? 0.0 : ub - delta, b0 = ub + delta > 1.0 ? 1.0 : ub + delta;
    if (b0 > a0) ns_panel(s, xs, a0, b0, R, acc);
    // left panels
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
    const double g4 = gamma[fil[sg]] / (4.0 * kPi);
    // subtract the Q-point sum the method used for this segment and image
    double qs[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        const double *qp = qpos + 3 * ((size_t)sg * Q + i), *qc = qchg + 3 * ((size_t)sg * Q + i);
        double r[3] = {qp[0] - xs[0], qp[1] - xs[1], qp[2] - xs[2]};
        double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        double f = 1.0 / (rr2 * sqrt(rr2));
        qs[0] += f * (r[1] * qc[2] - r[2] * qc[1]);
        qs[1] += f * (r[2] * qc[0] - r[0] * qc[2]);
        qs[2] += f * (r[0] * qc[1] - r[1] * qc[0]);
    }
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
    hipLaunchKernelGGL(k_max_ell, dim3(1), dim3(256), 0, p->stream, N,
                       (const double *)p->d_ell.p, (double *)p->ns_maxell.p);
    NsArgs a = ns_args(p);
    int *cnt = (int *)p->ns_cnt.p, *start = (int *)p->ns_start.p;
    hipLaunchKernelGGL((k_ns_flag<0>), grid, block, 0, p->stream, a, cnt, (const int *)nullptr,
                       (int2 *)nullptr, (int *)p->d_status.p);
    exclusive_scan(p, cnt, start, N);
    hipLaunchKernelGGL((k_ns_flag<1>), grid, block, 0, p->stream, a, (int *)nullptr, start,
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

}  // namespace bs
