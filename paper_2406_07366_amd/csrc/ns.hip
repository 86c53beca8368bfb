// Near-singular correction (not in the paper; the paper notes that the
// Q-point rule degrades for close segments and subdivides only the local
// ones, Sec. 5.2).  For every node i and every segment j that is not one of
// the two segments adjacent to i and whose chord passes closer to s_i than
// ns_eta * ell_j, the Q-point sum of segment j is replaced by the integral of
// the full Biot-Savart kernel over the spline segment:
//   dv_i += (Gamma_j/4pi) int_seg (s - s_i) x ds / |s - s_i|^3  -  sum_Q(...)
// (the same image of the segment as the chord test, minimum image).
//
// Passes (no host synchronisation):
//   search  segments binned by chord midpoint, targets by node cell; one
//           workgroup per target cell tests the window's segments and writes
//           each node's flagged pairs in a fixed order; compacted pair list;
//   integrate  one thread per pair, float64, by one of
//           - graded panels: closest point of the segment to the target by
//             Newton steps, 10-point (cubic) or 12-point (quintic)
//             Gauss-Legendre panels graded geometrically (ratio 3) away
//             from it (error ~1e-11 relative);
//           - the mapped rule: sinh-mapped 16-point rules on either side of
//             the closest point, the tangent segment as a control variate
//             (fixed cost);
//           - the learned correction where its error indicator allows (the
//             network runs only on those pairs), the graded panels elsewhere;
//   apply   one thread per node adds its pairs' corrections in list order
//           (deterministic whatever order the pairs were computed in).
#include <mutex>

#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

constexpr int kNsGL = 16;        // mapped rule, each side of the peak
struct NsRule {
    double x[kNsGL];   // nodes on [-1, 1]
    double w[kNsGL];
    double x10[10], w10[10];   // graded panels, cubic segments
    double x12[12], w12[12];   // graded panels, quintic segments
};

// ------------------------------------------------------------ cell grid
// A segment j flags target x when the distance from x to its chord is below
// eta * ell_j.  Then |x - m_j| < reach_j = eta * ell_j + |B_j - A_j| / 2 (m_j
// the chord midpoint), so with segments binned by midpoint into cells of edge
// >= max_j reach_j, every segment a target flags lies in the 3^3 cells around
// the target.  The cell count is decided on the device from that maximum.
constexpr int kNsRedBlocks = 1024;

// x: nodes; xn: end node of each segment in the segment's own frame
__global__ void k_ns_reach(int N, const double *__restrict__ x, const double *__restrict__ xn,
                           const double *__restrict__ ell, double eta,
                           double *__restrict__ pmax, double *__restrict__ psum) {
    __shared__ double sh[256], ss[256];
    double m = 0.0, sum = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
        double c2 = 0.0;
        for (int q = 0; q < 3; q++) {
            double d = xn[3 * j + q] - x[3 * j + q];
            c2 += d * d;
        }
        const double r = eta * ell[j] + 0.5 * sqrt(c2);
        m = fmax(m, r);
        sum += r;
    }
    sh[threadIdx.x] = m;
    ss[threadIdx.x] = sum;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
            ss[threadIdx.x] += ss[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pmax[blockIdx.x] = sh[0];
        psum[blockIdx.x] = ss[0];
    }
}

// Two cell grids for the segments.  Grid A, of nc_A = floor(L / h) cells per
// axis with h = min(max reach, 2 x mean reach) (at most ncmax), holds the
// short segments (reach <= L / nc_A): a target scans the 27 A-cells around
// its own.  Grid B, of nc_B = floor(L / max reach) cells, holds the few long
// ones (its cells are at least as large as any reach): a target cell scans
// the 4 x 4 x 4 B-cells from the B-cell of its lower corner minus one B edge.
// nc_A < 3: one A-cell holds every segment (and grid B is empty); nc_B < 4:
// one B-cell.  ncp[0] = nc_A, ncp[1] = nc_B.
__global__ void k_ns_cells(const double *__restrict__ pmax, const double *__restrict__ psum,
                           int nparts, int N, double L, int ncmax, double *__restrict__ maxreach,
                           int *__restrict__ ncp) {
    __shared__ double sh[256], ss[256];
    double m = 0.0, sum = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        m = fmax(m, pmax[i]);
        sum += psum[i];
    }
    sh[threadIdx.x] = m;
    ss[threadIdx.x] = sum;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
            ss[threadIdx.x] += ss[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        m = sh[0];
        const double mean = N > 0 ? ss[0] / N : 0.0;
        const double h = fmin(m, 2.0 * mean);
        double f = h > 0.0 ? floor(L / (h * (1.0 + 1e-9))) : (double)ncmax;
        int na = f > (double)ncmax ? ncmax : (int)f;
        if (na < 3) na = 1;
        f = m > 0.0 ? floor(L / (m * (1.0 + 1e-9))) : 1.0;
        int nb = f > (double)na ? na : (int)f;
        if (nb < 4 || na == 1) nb = 1;
        *maxreach = m;
        ncp[0] = na;
        ncp[1] = nb;
    }
}

__device__ __forceinline__ int cell_of(double v, double L, int nc) {
    int c = (int)(wrap_box(v, L) / L * nc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_ns_zero(int n, int *__restrict__ a, int *__restrict__ b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { a[i] = 0; b[i] = 0; }
}

// segment key: A-cell of the chord midpoint (short segments) or nc_A^3 +
// B-cell of the chord midpoint (long ones); target key: A-cell of the node
__global__ void k_ns_keys(int N, const double *__restrict__ x, const double *__restrict__ xn,
                          const double *__restrict__ ell, double eta,
                          double L, const int *__restrict__ ncp, int *__restrict__ key,
                          int *__restrict__ cnt, int *__restrict__ tkey, int *__restrict__ tcnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = j < N;
    int k = 0, kt = 0;
    if (valid) {
        const int na = ncp[0], nb = ncp[1];
        double c2 = 0.0, mid[3];
        int d[3];
        for (int q = 0; q < 3; q++) {
            const double e = xn[3 * j + q] - x[3 * j + q];
            c2 += e * e;
            mid[q] = 0.5 * (x[3 * j + q] + xn[3 * j + q]);
            d[q] = cell_of(x[3 * j + q], L, na);
        }
        const bool shortseg = na == 1 || eta * ell[j] + 0.5 * sqrt(c2) <= L / na;
        const int nc = shortseg ? na : nb;
        int c[3];
        for (int q = 0; q < 3; q++) c[q] = cell_of(mid[q], L, nc);
        k = (c[2] * nc + c[1]) * nc + c[0] + (shortseg ? 0 : na * na * na);
        key[j] = k;
        kt = (d[2] * na + d[1]) * na + d[0];
        tkey[j] = kt;
    }
    wave_add<false>(cnt, k, valid);
    wave_add<false>(tcnt, kt, valid);
}

// segments and targets into their cells (the order of targets within a cell
// does not matter; segments are ordered afterwards)
__global__ void k_ns_scatter(int N, const int *__restrict__ key, const int *__restrict__ start,
                             int *__restrict__ fill, int *__restrict__ perm,
                             const int *__restrict__ tkey, const int *__restrict__ tstart,
                             int *__restrict__ tfill, int *__restrict__ tperm) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = j < N;
    const int k = valid ? key[j] : 0, kt = valid ? tkey[j] : 0;
    // both atomics of a group leader in flight together
    const WaveGroup g = wave_group(k, 0, valid), gt = wave_group(kt, 0, valid);
    const int lane = threadIdx.x & 63;
    int o = 0, ot = 0;
    if (valid && lane == g.leader) o = atomicAdd(fill + k, g.size);
    if (valid && lane == gt.leader) ot = atomicAdd(tfill + kt, gt.size);
    const int r = __shfl(o, g.leader) + g.rank, rt = __shfl(ot, gt.leader) + gt.rank;
    if (valid) {
        perm[start[k] + r] = j;
        tperm[tstart[kt] + rt] = j;
    }
}

// one wavefront per occupied cell range, striding over the nc^3 cells
constexpr int kNsSortLds = 1024;
__global__ __launch_bounds__(64) void k_ns_sort(const int *__restrict__ ncp,
                                               const int *__restrict__ start, int *__restrict__ perm,
                                               int *__restrict__ scratch) {
    __shared__ int v[kNsSortLds];
    const int na = ncp[0], nbb = ncp[1], nb = na * na * na + nbb * nbb * nbb;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int s0 = start[b], n = start[b + 1] - s0;
        rank_sort_bin<kNsSortLds>(perm, scratch, s0, n, v);
        __syncthreads();
    }
}

// period index of v (floor(v / L), clamped to +-511) and v wrapped into the
// box by it; kept consistent so that v = w + L k up to rounding
__device__ __forceinline__ int period_of(double v, double L, double *w) {
    double k = floor(v / L);
    k = k < -511.0 ? -511.0 : (k > 511.0 ? 511.0 : k);
    *w = v - L * k;
    return (int)k;
}
__device__ __forceinline__ int pack_periods(const int *k) {
    return ((k[0] + 512) << 20) | ((k[1] + 512) << 10) | (k[2] + 512);
}

// cell-ordered copies of each segment's end points, weight ell and index,
// and the float32 capsule of the flag test: chord midpoint moved into the
// box and eta ell (segM), half chord and the midpoint's packed period
// indices (segH)
__global__ void k_ns_gather(int N, const int *__restrict__ perm, const double *__restrict__ x,
                            const double *__restrict__ xn,
                            const double *__restrict__ ell, double eta, double L,
                            double4 *__restrict__ segA, double4 *__restrict__ segB,
                            float4 *__restrict__ segM, float4 *__restrict__ segH) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int j = perm[p];
    segA[p] = make_double4(x[3 * j], x[3 * j + 1], x[3 * j + 2], ell[j]);
    segB[p] = make_double4(xn[3 * j], xn[3 * j + 1], xn[3 * j + 2], (double)j);
    double m[3], h[3];
    int k[3];
    for (int q = 0; q < 3; q++) {
        h[q] = 0.5 * (xn[3 * j + q] - x[3 * j + q]);
        k[q] = period_of(0.5 * (x[3 * j + q] + xn[3 * j + q]), L, &m[q]);
    }
    // a midpoint beyond the clamped period range gets a negative eta ell,
    // which sends every test against it to the float64 decision
    const bool clamped = abs(k[0]) == 511 || abs(k[1]) == 511 || abs(k[2]) == 511;
    segM[p] = make_float4((float)m[0], (float)m[1], (float)m[2],
                          clamped ? -1.f : (float)(eta * ell[j]));
    segH[p] = make_float4((float)h[0], (float)h[1], (float)h[2],
                          __int_as_float(pack_periods(k)));
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
    int N, max_per_node;
    double L, eta;
    const double *x;
    const int *off, *fil, *ncp, *cstart, *segj;
    const double4 *segA, *segB;
    const float4 *segM, *segH;
};

// Target of a flag test: the node, its previous node (the two adjacent
// segments are excluded), its position in float32 moved into the box with
// its period indices (packed as in segH); exact: beyond the clamped period
// range, every test in float64.
struct NsTarget {
    int o, ip, kp;
    bool exact;
    float xf[3];
};

__device__ __forceinline__ NsTarget ns_target(const NsArgs &a, int o) {
    NsTarget T;
    T.o = o;
    T.ip = prev_node_d(a.off, a.fil, o);
    int k[3];
    for (int q = 0; q < 3; q++) {
        double w;
        k[q] = period_of(a.x[3 * o + q], a.L, &w);
        T.xf[q] = (float)w;
    }
    T.kp = pack_periods(k);
    T.exact = abs(k[0]) == 511 || abs(k[1]) == 511 || abs(k[2]) == 511;
    return T;
}

// The float64 decision: chord distance < eta * ell for segment record p
// (cell order); on success the segment index and the target's image shift,
// periods per axis packed as three 10-bit fields (+-511 periods).
__device__ __forceinline__ bool ns_test_exact(const NsArgs &a, const NsTarget &T, int p,
                                           int *sg_out, int *sh_out) {
    const double4 A4 = a.segA[p], B4 = a.segB[p];
    const int sg = (int)B4.w;
    if (sg == T.o || sg == T.ip) return false;
    const double A[3] = {A4.x, A4.y, A4.z}, Bv[3] = {B4.x, B4.y, B4.z};
    const double x[3] = {a.x[3 * T.o], a.x[3 * T.o + 1], a.x[3 * T.o + 2]};
    double xs[3];
    if (!(chord_dist(A, Bv, x, a.L, xs) < a.eta * A4.w)) return false;
    int sh = 0;
    for (int q = 0; q < 3; q++) {
        int sv = (int)rint((xs[q] - x[q]) / a.L);
        sv = sv < -511 ? -511 : (sv > 511 ? 511 : sv);
        sh = (sh << 10) | (sv + 512);
    }
    *sg_out = sg;
    *sh_out = sh;
    return true;
}

// Does segment record p flag target T?  The capsule test in float32: the
// distance from the target to the chord (midpoint M4, half chord H4, minimum
// image of the midpoint) against eta ell (M4.w).  Both points carry at most a
// few 1e-8 L of rounding, so a distance more than 1e-5 L inside or outside
// the capsule decides as the float64 test would; the band between, and
// targets near half a period from the midpoint (where the image could
// differ), go to the float64 test.  An accepted target's image shift follows
// from the period indices: the float64 test shifts the target by
// -rint((x - m) / L) periods, and x - m = (x_box - m_box) + L (k_x - k_m).
__device__ __forceinline__ bool ns_test(const NsArgs &a, const NsTarget &T, float4 M4, float4 H4,
                                        int p, int *sg_out, int *sh_out) {
    const float Lf = (float)a.L, iLf = (float)(1.0 / a.L), band = (float)(1e-5 * a.L);
    float d[3], w[3], far = 0.f;
    const float m[3] = {M4.x, M4.y, M4.z}, h[3] = {H4.x, H4.y, H4.z};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const float t = (T.xf[q] - m[q]) * iLf;
        w[q] = rintf(t);
        far = fmaxf(far, fabsf(t - w[q]));
        d[q] = fmaf(-Lf, w[q], T.xf[q] - m[q]);
    }
    const float hh = h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
    float u = (d[0] * h[0] + d[1] * h[1] + d[2] * h[2]) * __builtin_amdgcn_rcpf(hh);
    u = hh > 0.f ? fminf(fmaxf(u, -1.f), 1.f) : 0.f;
    float r2 = 0.f;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const float e = fmaf(-u, h[q], d[q]);
        r2 = fmaf(e, e, r2);
    }
    const float lo = M4.w - band, hi = M4.w + band;
    if (!(lo > 0.f) || far > 0.45f || T.exact) return ns_test_exact(a, T, p, sg_out, sh_out);
    if (r2 >= hi * hi) return false;
    if (r2 > lo * lo) return ns_test_exact(a, T, p, sg_out, sh_out);
    const int sg = a.segj[p];
    if (sg == T.o || sg == T.ip) return false;
    const int km = __float_as_int(H4.w);
    int sh = 0;
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int sh_q = 20 - 10 * q;
        int sv = -(((T.kp >> sh_q) & 1023) - ((km >> sh_q) & 1023) + (int)w[q]);
        sv = sv < -511 ? -511 : (sv > 511 ? 511 : sv);
        sh = (sh << 10) | (sv + 512);
    }
    *sg_out = sg;
    *sh_out = sh;
    return true;
}

// Necessary condition for ns_test to accept: a target within eta ell of
// the chord lies within eta ell + |half chord| of the chord midpoint's
// nearest image.  The staged midpoint m is that image for every target of
// the cell (section below), r2m = (|h| + eta ell + 1e-5 L)^2 (the margin
// covers the float32 rounding of both points), infinite for records that
// every target passes.
__device__ __forceinline__ bool ns_pretest(const float *xf, float4 M4, float r2m) {
    const float d0 = xf[0] - M4.x, d1 = xf[1] - M4.y, d2 = xf[2] - M4.z;
    return fmaf(d2, d2, fmaf(d1, d1, d0 * d0)) < r2m;
}

// Lanes 0..26 of a wavefront: start and size of one of the 27 cells around
// cell (c0x, c0y, c0z) (lane 0: the single cell when nc < 3); returns the
// lane's exclusive prefix of the sizes and the total in *total.
__device__ __forceinline__ int ns_window(const NsArgs &a, int nc, const int *c0, int lane,
                                         int *cs, int *cn, int *total) {
    const int ncell = nc >= 3 ? 27 : 1;
    *cs = 0; *cn = 0;
    if (lane < ncell) {
        int cidx = 0;
        if (nc >= 3) {
            const int dd[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
            int c[3];
            for (int q = 0; q < 3; q++) {
                int v = c0[q] + dd[q];
                c[q] = v < 0 ? v + nc : (v >= nc ? v - nc : v);
            }
            cidx = (c[2] * nc + c[1]) * nc + c[0];
        }
        *cs = a.cstart[cidx];
        *cn = a.cstart[cidx + 1] - *cs;
    }
    int incl = *cn;
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    *total = __shfl(incl, 63);
    return incl - *cn;
}

// Used when fewer than 3 cells fit along an axis (one cell holds every
// segment): one wavefront per target, 64 candidates per step, flagged ones
// ranked with a ballot and written in candidate order to the target's
// max_per_node slots.
__global__ __launch_bounds__(256) void k_ns_flag(NsArgs a, int *__restrict__ cnt,
                                                 int2 *__restrict__ slots,
                                                 int *__restrict__ status) {
    if (*a.ncp >= 3) return;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = gid & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int t = gid >> 6; t < a.N; t += (gridDim.x * blockDim.x) >> 6) {
        const NsTarget T = ns_target(a, t);
        const int zero[3] = {0, 0, 0};
        int cs, cn, total;
        ns_window(a, 1, zero, lane, &cs, &cn, &total);
        const int s0 = __shfl(cs, 0);
        int2 *out = slots + (size_t)T.o * a.max_per_node;
        int k = 0;
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            int sg = 0, sh = 0;
            const bool flag =
                q < total && ns_test(a, T, a.segM[s0 + q], a.segH[s0 + q], s0 + q, &sg, &sh);
            const unsigned long long m = __ballot(flag);
            if (flag) {
                const int slot = k + __popcll(m & below);
                if (slot < a.max_per_node) out[slot] = make_int2(sg, sh);
            }
            k += __popcll(m);
        }
        if (lane == 0) {
            if (k > a.max_per_node) atomicOr(status, 2);
            cnt[T.o] = k < a.max_per_node ? k : a.max_per_node;
        }
    }
}

// One workgroup per cell of targets (nc >= 3).  The segment records of the
// 27 cells around it (cell order, then segment order) are staged in LDS in
// chunks of kNsStage and shared by every target of the cell; wavefront w
// takes targets w, w + 4, ...  and scans each chunk 64 candidates per step.
// Flagged candidates are ranked with a ballot, so each target's pairs are
// written in candidate order to its max_per_node slots.  Targets are taken
// 256 at a time (their running counts live in LDS).  A cheap sphere test
// (ns_pretest) runs first on every candidate; the ~3 % that pass it are
// queued per wavefront, in candidate order, and the capsule test runs on
// the queue 64 at a time, so the order of each target's pairs is that of
// the full scan.  Records of 40 B (two float4 capsules, the sphere radius
// and the index), 512 at a time, and at most 96 VGPRs keep five wavefronts
// per SIMD.
constexpr int kNsStage = 512;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_ns_flag_cells(NsArgs a, const int *__restrict__ tstart,
                                                       const int *__restrict__ tperm,
                                                       int *__restrict__ cnt,
                                                       int2 *__restrict__ slots,
                                                       int *__restrict__ status) {
    __shared__ float4 sm[kNsStage], sh4[kNsStage];
    __shared__ int sp[kNsStage];
    __shared__ float sr2[kNsStage];
    __shared__ short sq[4][128];   // per wavefront: queued candidates
    // window: the 27 A-cells (entries 0..26), then the B-cells (27..90)
    constexpr int kWin = 27 + 64;
    __shared__ int cell_s[kWin], cell_o[kWin], tk[256], tot_a, tot_b;
    __shared__ int t_o[256], t_ip[256], t_kp[256];   // targets of the group (kp bit 30: exact)
    __shared__ float t_xf[3][256];
    const int nc = a.ncp[0], ncb = a.ncp[1];
    if (nc < 3) return;
    const int nb3 = nc * nc * nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float Lf = (float)a.L, iLf = (float)(1.0 / a.L), band = (float)(1e-5 * a.L);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int C = blockIdx.x; C < nb3; C += gridDim.x) {
        const int t0 = tstart[C], nt = tstart[C + 1] - t0;
        if (nt == 0) continue;   // uniform over the workgroup
        const int c0[3] = {C % nc, (C / nc) % nc, C / (nc * nc)};
        const float cc[3] = {(float)((c0[0] + 0.5) * a.L / nc), (float)((c0[1] + 0.5) * a.L / nc),
                             (float)((c0[2] + 0.5) * a.L / nc)};   // the cell's centre
        if (wave == 0) {
            int cs, cn, total;
            const int excl = ns_window(a, nc, c0, lane, &cs, &cn, &total);
            if (lane < 27) { cell_s[lane] = cs; cell_o[lane] = excl; }
            if (lane == 0) tot_a = total;
        } else if (wave == 1) {
            // B-cells: 4 per axis from the B-cell of (lower corner - B edge),
            // or the single B-cell
            int cs = 0, cn = 0;
            if (ncb >= 4 || lane == 0) {
                int cidx = 0;
                if (ncb >= 4) {
                    const double ha = a.L / nc, hb = a.L / ncb;
                    const int dd[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
                    int c[3];
                    for (int q = 0; q < 3; q++) {
                        int v = (int)floor((c0[q] * ha - hb) / hb) + dd[q];
                        v %= ncb;
                        c[q] = v < 0 ? v + ncb : v;
                    }
                    cidx = (c[2] * ncb + c[1]) * ncb + c[0];
                }
                cidx += nb3;
                cs = a.cstart[cidx];
                cn = a.cstart[cidx + 1] - cs;
            }
            int incl = cn;
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl, d);
                if (lane >= d) incl += v;
            }
            cell_s[27 + lane] = cs;
            cell_o[27 + lane] = incl - cn;   // relative; tot_a added below
            if (lane == 63) tot_b = incl;
        }
        __syncthreads();
        if (threadIdx.x < 64) cell_o[27 + threadIdx.x] += tot_a;
        __syncthreads();
        const int total = tot_a + tot_b;
        for (int g0 = 0; g0 < nt; g0 += 256) {
            const int ng = nt - g0 < 256 ? nt - g0 : 256;
            // each target's flag-test data, once (one thread per target; the
            // chunk loop below reads it from LDS)
            for (int i = threadIdx.x; i < ng; i += blockDim.x) {
                const NsTarget T = ns_target(a, tperm[t0 + g0 + i]);
                tk[i] = 0;
                t_o[i] = T.o;
                t_ip[i] = T.ip;
                t_kp[i] = T.kp | (T.exact ? 1 << 30 : 0);
                t_xf[0][i] = T.xf[0]; t_xf[1][i] = T.xf[1]; t_xf[2][i] = T.xf[2];
            }
            for (int c0 = 0; c0 < total; c0 += kNsStage) {
                const int cn = total - c0 < kNsStage ? total - c0 : kNsStage;
                for (int i = threadIdx.x; i < cn; i += blockDim.x) {
                    const int q = c0 + i;
                    int c = 0;
                    for (int step = 64; step > 0; step >>= 1) {
                        const int tc = c + step;
                        if (tc < kWin && cell_o[tc] <= q) c = tc;
                    }
                    const int p = cell_s[c] + (q - cell_o[c]);
                    float4 M4 = a.segM[p], H4 = a.segH[p];
                    // the midpoint's image nearest the cell's centre, with its
                    // period indices moved by the same shift (the capsule
                    // test's float decision and image shift are unchanged):
                    // for every target of the cell that is the nearest image
                    // when the window lies within 0.45 L of the cell
                    // (window A: 2 h_A, five or more cells per axis; window
                    // B: 3 h_B, eight or more).  Other records, and midpoints
                    // beyond the clamped period range (negative eta ell, sent
                    // to the float64 decision), pass every target.
                    float r2m = INFINITY;
                    if ((q < tot_a ? nc >= 5 : ncb >= 8) && M4.w >= 0.f) {
                        int km = __float_as_int(H4.w);
                        float m[3] = {M4.x, M4.y, M4.z};
#pragma unroll
                        for (int ax = 0; ax < 3; ax++) {
                            const float sft = rintf((cc[ax] - m[ax]) * iLf);
                            m[ax] = fmaf(Lf, sft, m[ax]);
                            km -= (int)sft * (1 << (20 - 10 * ax));
                        }
                        M4.x = m[0]; M4.y = m[1]; M4.z = m[2];
                        H4.w = __int_as_float(km);
                        const float r = sqrtf(H4.x * H4.x + H4.y * H4.y + H4.z * H4.z) + M4.w + band;
                        r2m = r * r;
                    }
                    sm[i] = M4;
                    sh4[i] = H4;
                    sp[i] = p;
                    sr2[i] = r2m;
                }
                __syncthreads();
                for (int ti = wave; ti < ng; ti += 4) {
                    NsTarget T;
                    T.o = t_o[ti];
                    T.ip = t_ip[ti];
                    T.kp = t_kp[ti] & ((1 << 30) - 1);
                    T.exact = (t_kp[ti] >> 30) & 1;
                    T.xf[0] = t_xf[0][ti]; T.xf[1] = t_xf[1][ti]; T.xf[2] = t_xf[2][ti];
                    int2 *out = slots + (size_t)T.o * a.max_per_node;
                    int k = tk[ti];
                    short *qw = sq[wave];
                    // capsule test on the first nq (<= 64) queued candidates
                    auto drain = [&](int nq) {
                        const int j = lane < nq ? qw[lane] : 0;
                        int sg = 0, sh = 0;
                        const bool flag =
                            lane < nq && ns_test(a, T, sm[j], sh4[j], sp[j], &sg, &sh);
                        const unsigned long long m = __ballot(flag);
                        if (flag) {
                            const int slot = k + __popcll(m & below);
                            if (slot < a.max_per_node) out[slot] = make_int2(sg, sh);
                        }
                        k += __popcll(m);
                    };
                    // pre-test 64 candidates per step while any are left; drain
                    // the queue when it holds 64, and to the end after the last
                    int nq = 0;
                    for (int j0 = 0;;) {
                        if (j0 < cn) {
                            const int j = j0 + lane;
                            const bool pass =
                                j < cn && (T.exact || ns_pretest(T.xf, sm[j], sr2[j]));
                            const unsigned long long m = __ballot(pass);
                            if (pass) qw[nq + __popcll(m & below)] = (short)j;
                            nq += __popcll(m);
                            j0 += 64;
                        }
                        const bool done = j0 >= cn;
                        if (nq >= 64 || (done && nq > 0)) {
                            const int d = nq < 64 ? nq : 64;
                            drain(d);
                            const short rest = lane < nq - d ? qw[d + lane] : (short)0;
                            if (lane < nq - d) qw[lane] = rest;
                            nq -= d;
                        }
                        if (done && nq == 0) break;
                    }
                    if (lane == 0) tk[ti] = k;
                }
                __syncthreads();
            }
            for (int i = threadIdx.x; i < ng; i += blockDim.x) {
                const int o = t_o[i], k = tk[i];
                if (k > a.max_per_node) atomicOr(status, 2);
                cnt[o] = k < a.max_per_node ? k : a.max_per_node;
            }
            __syncthreads();
        }
    }
}

// compact list: node o's pairs at [start[o], start[o] + cnt[o]), owner
// pnode; kNsCompactLanes lanes per node step through its used slots only
constexpr int kNsCompactLanes = 16;
__global__ void k_ns_compact(int N, int maxpn, const int *__restrict__ cnt,
                             const int *__restrict__ start, const int2 *__restrict__ slots,
                             int2 *__restrict__ pairs, int *__restrict__ pnode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int o = (int)(i / kNsCompactLanes);
    if (o >= N) return;
    const int n = cnt[o], b = start[o];
    for (int s = (int)(i % kNsCompactLanes); s < n; s += kNsCompactLanes) {
        pairs[b + s] = slots[(size_t)o * maxpn + s];
        pnode[b + s] = o;
    }
}

// spline segment j as c0 + c1 u + ... + c5 u^5, u in [0, 1]: the cubic
// Hermite segment (c4 = c5 = 0) from node values and slopes, or, when the
// nodal second derivatives S are given, the quintic Hermite segment; the
// derivative's coefficients k c_k are kept beside them (e2 = 2 c2, ...)
struct Seg {
    double c0[3], c1[3], c2[3], c3[3], c4[3], c5[3];
    double e2[3], e3[3], e4[3], e5[3];
};

// the derivative's coefficients from c0 .. c5 (every Seg is finished by it)
__device__ __forceinline__ void seg_derivs(Seg &s) {
    for (int q = 0; q < 3; q++) {
        s.e2[q] = 2.0 * s.c2[q];
        s.e3[q] = 3.0 * s.c3[q];
        s.e4[q] = 4.0 * s.c4[q];
        s.e5[q] = 5.0 * s.c5[q];
    }
}

// (from node j to xn[j], its end node in the segment's own frame)
__device__ __forceinline__ Seg load_seg(int j, const int *off, const int *fil, const double *x,
                                        const double *xn, const double *D, const double *S,
                                        const double *dtau) {
    Seg s;
    int jn = next_node_d(off, fil, j);
    double h = dtau[j];
    for (int q = 0; q < 3; q++) {
        double s0 = x[3 * j + q], s1 = xn[3 * j + q];
        double d0 = h * D[3 * j + q], d1 = h * D[3 * jn + q];
        s.c0[q] = s0;
        s.c1[q] = d0;
        if (S) {
            const double q0 = h * h * S[3 * j + q], q1 = h * h * S[3 * jn + q];
            const double A = s1 - s0 - d0 - 0.5 * q0, B = d1 - d0 - q0, C = q1 - q0;
            s.c2[q] = 0.5 * q0;
            s.c3[q] = 10.0 * A - 4.0 * B + 0.5 * C;
            s.c4[q] = -15.0 * A + 7.0 * B - C;
            s.c5[q] = 6.0 * A - 3.0 * B + 0.5 * C;
        } else {
            s.c2[q] = 3.0 * (s1 - s0) - 2.0 * d0 - d1;
            s.c3[q] = 2.0 * (s0 - s1) + d0 + d1;
            s.c4[q] = s.c5[q] = 0.0;
        }
    }
    seg_derivs(s);
    return s;
}

// component q of s(u), s'(u), s''(u); DEG = 3 leaves out the terms that
// vanish on cubic segments (the same values: a zero term adds exactly 0)
template <int DEG = 5>
__device__ __forceinline__ double seg_p(const Seg &s, int q, double u) {
    if constexpr (DEG == 3) return s.c0[q] + u * (s.c1[q] + u * (s.c2[q] + u * s.c3[q]));
    return s.c0[q] + u * (s.c1[q] + u * (s.c2[q] + u * (s.c3[q] + u * (s.c4[q] + u * s.c5[q]))));
}
template <int DEG = 5>
__device__ __forceinline__ double seg_d(const Seg &s, int q, double u) {
    if constexpr (DEG == 3) return s.c1[q] + u * (s.e2[q] + u * s.e3[q]);
    return s.c1[q] + u * (s.e2[q] + u * (s.e3[q] + u * (s.e4[q] + u * s.e5[q])));
}
template <int DEG = 5>
__device__ __forceinline__ double seg_dd(const Seg &s, int q, double u) {
    if constexpr (DEG == 3) return s.e2[q] + u * 2.0 * s.e3[q];
    return s.e2[q] + u * (2.0 * s.e3[q] + u * (3.0 * s.e4[q] + u * 4.0 * s.e5[q]));
}

// 1 / sqrt(a) for a > 0: the hardware estimate and two Newton steps
// y <- y (3 - a y^2) / 2 (each squares the relative error), to rounding
__device__ __forceinline__ double rsqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// integral over u in [a, b] of (s(u) - x) x s'(u) / |s(u) - x|^3 by
// Gauss-Legendre: 10 points on cubic segments, 12 on quintic ones.  On the
// graded panels below, the integrand's complex singularity near the closest
// point (2 delta off the real axis) lies outside the Bernstein ellipse of
// parameter 3.7 of every panel (4.2 for the centre panel; clipped panels
// only shrink), so the rule's relative error is of order 3.7^-20 = 4e-12 at
// 10 points (measured on cubic segments against the oracle's adaptive
// Gauss-Kronrod: 9e-12; 12 points gave 2e-13 for 13 % more time).  Quintic
// segments, whose |s(u) - x|^2 has more complex roots, measured 8e-10 at 10
// points and 7e-13 at 12, so they keep 12.
template <int DEG = 5>
__device__ void ns_panel(const Seg &s, const double *x, double a, double b, const NsRule &R,
                         double *acc) {
    constexpr int NG = DEG == 3 ? 10 : 12;
    const double *gx = DEG == 3 ? R.x10 : R.x12, *gw = DEG == 3 ? R.w10 : R.w12;
    double m = 0.5 * (a + b), hw = 0.5 * (b - a);
    for (int k = 0; k < NG; k++) {
        double u = m + hw * gx[k];
        double r[3], d[3];
        for (int q = 0; q < 3; q++) {
            r[q] = seg_p<DEG>(s, q, u) - x[q];
            d[q] = seg_d<DEG>(s, q, u);
        }
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double y = rsqrt_nr(r2);
        const double f = gw[k] * hw * (y * y * y);
        acc[0] += f * (r[1] * d[2] - r[2] * d[1]);
        acc[1] += f * (r[2] * d[0] - r[0] * d[2]);
        acc[2] += f * (r[0] * d[1] - r[1] * d[0]);
    }
}

// Integral over u in [0,1] of (s(u) - x) x s'(u) / |s(u) - x|^3 for one
// cubic segment: closest point by a coarse scan and Newton steps on
// (s - x) . s' = 0, then Gauss-Legendre panels graded geometrically (ratio
// 3) away from it.
template <int DEG = 5>
__device__ __forceinline__ void seg_eval(const Seg &s, double u, double *p, double *d1) {
    for (int q = 0; q < 3; q++) {
        p[q] = seg_p<DEG>(s, q, u);
        d1[q] = seg_d<DEG>(s, q, u);
    }
}

// parameter of the point of the segment closest to x: best of a coarse scan,
// then Newton steps on (s - x) . s' = 0 kept inside [0, 1], until a step
// moves u by less than 1e-14
template <int DEG = 5>
__device__ double closest_u(const Seg &s, const double *xs) {
    double ub = 0.0, best = 1e300;
    for (int k = 0; k <= 8; k++) {
        double u = k / 8.0, r2 = 0.0;
        for (int q = 0; q < 3; q++) {
            double r = seg_p<DEG>(s, q, u) - xs[q];
            r2 += r * r;
        }
        if (r2 < best) { best = r2; ub = u; }
    }
    for (int it = 0; it < 8; it++) {
        double g = 0.0, dg = 0.0;
        for (int q = 0; q < 3; q++) {
            double r = seg_p<DEG>(s, q, ub) - xs[q];
            double d1 = seg_d<DEG>(s, q, ub);
            double d2 = seg_dd<DEG>(s, q, ub);
            g += r * d1;
            dg += d1 * d1 + r * d2;
        }
        if (!(dg > 0.0)) break;
        double un = ub - g / dg;
        un = un < 0.0 ? 0.0 : (un > 1.0 ? 1.0 : un);
        const bool done = fabs(un - ub) < 1e-14;
        ub = un;
        if (done) break;
    }
    return ub;
}

template <int DEG = 5>
__device__ void ns_seg_integral(const Seg &s, const double *xs, const NsRule &R, double *acc) {
    const double ub = closest_u<DEG>(s, xs);
    double P[3], d1[3];
    seg_eval<DEG>(s, ub, P, d1);
    const double r2 = (P[0] - xs[0]) * (P[0] - xs[0]) + (P[1] - xs[1]) * (P[1] - xs[1]) +
                      (P[2] - xs[2]) * (P[2] - xs[2]);
    const double sp2 = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    // half the distance in parameter units: the first panel pair is finer
    // than the singularity's width
    double delta = 0.5 * sqrt(r2 / sp2);
    delta = delta < 1e-13 ? 1e-13 : delta;
    acc[0] = acc[1] = acc[2] = 0.0;
    double a0 = ub - delta < 0.0 ? 0.0 : ub - delta, b0 = ub + delta > 1.0 ? 1.0 : ub + delta;
    if (b0 > a0) ns_panel<DEG>(s, xs, a0, b0, R, acc);
    double edge = a0, width = delta;
    while (edge > 0.0) {
        double nxt = ub - 3.0 * width;
        if (nxt < 0.0) nxt = 0.0;
        ns_panel<DEG>(s, xs, nxt, edge, R, acc);
        edge = nxt;
        width *= 3.0;
    }
    edge = b0; width = delta;
    while (edge < 1.0) {
        double nxt = ub + 3.0 * width;
        if (nxt > 1.0) nxt = 1.0;
        ns_panel<DEG>(s, xs, edge, nxt, R, acc);
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
        const double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double y = rsqrt_nr(rr2);
        const double f = y * y * y;
        qs[0] += f * (r[1] * qc[2] - r[2] * qc[1]);
        qs[1] += f * (r[2] * qc[0] - r[0] * qc[2]);
        qs[2] += f * (r[0] * qc[1] - r[1] * qc[0]);
    }
}

__device__ __forceinline__ void unpack_shift(int sh, const double *x, double L, double *xs) {
    int shv[3] = {((sh >> 20) & 1023) - 512, ((sh >> 10) & 1023) - 512, (sh & 1023) - 512};
    for (int q = 0; q < 3; q++) xs[q] = x[q] + shv[q] * L;
}

// Exact segment integral minus its Q-point sum, for one (node, segment) pair
// (DEG 3: cubic segments, S == NULL)
template <int DEG>
__device__ void ns_pair(int o, int sg, int sh, const int *off, const int *fil, const double *x,
                        const double *xn, const double *D, const double *S, const double *dtau, const double *gamma,
                        const double *qpos, const double *qchg, int Q, double L,
                        const NsRule &R, double *out) {
    double xs[3];
    unpack_shift(sh, x + 3 * o, L, xs);
    Seg s = load_seg(sg, off, fil, x, xn, D, S, dtau);
    double acc[3], qs[3];
    ns_seg_integral<DEG>(s, xs, R, acc);
    ns_qsum(sg, xs, qpos, qchg, Q, qs);
    const double g4 = gamma[fil[sg]] / (4.0 * kPi);
    for (int q = 0; q < 3; q++) out[q] = g4 * acc[q] - qs[q] / (4.0 * kPi);
}

// every pair (list == nullptr, count = total pairs), or the pairs listed.
// Held to 128 VGPRs (four wavefronts per SIMD instead of three at 158, no
// spills: 1.32 -> 1.27 ms for the 1.1e7 pairs of the 1e6-node tangle)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ns_integrate(
    const int *__restrict__ count, const int *__restrict__ list, const int *__restrict__ pnode,
    const int2 *__restrict__ pairs, const int *__restrict__ off, const int *__restrict__ fil,
    const double *__restrict__ x, const double *__restrict__ xn, const double *__restrict__ D,
    const double *__restrict__ S, const double *__restrict__ dtau,
    const double *__restrict__ gamma, const double *__restrict__ qpos,
    const double *__restrict__ qchg, int Q, double L, NsRule R, double *__restrict__ pout,
    const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int P = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const int p = list ? list[i] : i;
        int2 pr = pairs[p];
        double out[3];
        if (S)
            ns_pair<5>(pnode[p], pr.x, pr.y, off, fil, x, xn, D, S, dtau, gamma, qpos, qchg, Q, L,
                       R, out);
        else
            ns_pair<3>(pnode[p], pr.x, pr.y, off, fil, x, xn, D, S, dtau, gamma, qpos, qchg, Q, L,
                       R, out);
        pout[3 * (size_t)p] = out[0];
        pout[3 * (size_t)p + 1] = out[1];
        pout[3 * (size_t)p + 2] = out[2];
    }
}

// v[o] += the sum of node o's pair terms, in pair order.  The pairs of a
// workgroup's 256 nodes are one contiguous range of pout: it is staged
// through LDS in chunks with coalesced loads (a thread walking its own pairs
// in global memory touched a cache line per lane), and each node then sums
// its own pairs from LDS in the same order.  Launched with 256 threads.
constexpr int kNsApplyChunk = 1024;   // pairs per staged chunk (24 KB)
__global__ __launch_bounds__(256) void k_ns_apply(int N, const int *__restrict__ pstart,
                                                  const double *__restrict__ pout,
                                                  double *__restrict__ v) {
    __shared__ double sp[3 * kNsApplyChunk];
    const int o0 = blockIdx.x * 256, o = o0 + (int)threadIdx.x;
    if (o0 >= N) return;   // uniform over the workgroup
    const int oe = o0 + 256 < N ? o0 + 256 : N;
    const int p0 = pstart[o0], p1 = pstart[oe];
    int ps = 0, pe = 0;
    if (o < N) { ps = pstart[o]; pe = pstart[o + 1]; }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int c0 = p0; c0 < p1; c0 += kNsApplyChunk) {
        const int cn = p1 - c0 < kNsApplyChunk ? p1 - c0 : kNsApplyChunk;
        __syncthreads();   // the previous chunk's reads are done
        const double *src = pout + 3 * (size_t)c0;
        for (int i = threadIdx.x; i < 3 * cn; i += 256) sp[i] = src[i];
        __syncthreads();
        const int a = ps > c0 ? ps : c0, b = pe < c0 + cn ? pe : c0 + cn;
        for (int q = a - c0; q < b - c0; q++) {
            s0 += sp[3 * q];
            s1 += sp[3 * q + 1];
            s2 += sp[3 * q + 2];
        }
    }
    if (o < N) {
        v[3 * o] += s0;
        v[3 * o + 1] += s1;
        v[3 * o + 2] += s2;
    }
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

// Error indicator of the learned integral: err[b] is the root-mean-square
// error (raw integral, chord length h = 1) of the learned segment integral on
// held-out samples whose distance to the chord falls in bin b, measured
// against the plain method's graded-panel integrals (bs_ns_error_table).  A
// pair takes the network when err[b] |Gamma| / (4 pi h) sqrt(P / N) <= tol *
// v_scale: P pairs over N nodes add their errors to the nodes, so the rms
// velocity error they cause stays below tol times the velocity scale v_scale,
// the rms of the velocity's local, self and short-range terms at the nodes.
struct NsBox {
    float err[kNsBins];
    double tol;
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
// the same 1/d singularity as the curve (d = |P - x|), and the remainder
// I_seg - I_tan grows only like log(1/d) as d -> 0.  Returns I_tan (raw
// integral), the target multiplier mult = (1 + log(1 + h/d)) / h that
// bounds that remainder (the network predicts (I_seg - I_tan) / mult), the
// tangent segment's absolute integral S = int |ds| / |s - x|^2 in closed form
// (the scale errors are measured against; it never vanishes), and d/h.
struct TangentBase {
    double I[3];
    double mult, S, dstar;
};

__device__ TangentBase tangent_baseline(const Seg &s, const double *x, double h) {
    TangentBase tb;
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
    double A[3], B[3], t[3];
    for (int q = 0; q < 3; q++) {
        t[q] = d1[q] / tn;
        A[q] = P[q] - a * t[q];
        B[q] = P[q] + b * t[q];
    }
    chord_raw(A, B, x, tb.I);
    // int_0^len dl / (rho^2 + (l + p)^2) = atan2(rho len, rho^2 + u1 u2) / rho,
    // u1 = p, u2 = p + len, p = (A - x).t, rho the distance to the line
    double p = 0.0, r2 = 0.0;
    for (int q = 0; q < 3; q++) {
        p += (A[q] - x[q]) * t[q];
        r2 += (A[q] - x[q]) * (A[q] - x[q]);
    }
    const double len = a + b, u1 = p, u2 = p + len;
    double rho2 = r2 - p * p;
    rho2 = rho2 > 0.0 ? rho2 : 0.0;
    const double rho = sqrt(rho2);
    tb.S = rho > 1e-300 ? atan2(rho * len, rho2 + u1 * u2) / rho : len / (u1 * u2);
    tb.dstar = d / h;
    tb.mult = (1.0 + log1p(h / fmax(d, 1e-300 * h))) / h;
    return tb;
}

// ------------------------------------------------------ mapped rule
// Fixed-cost segment integral for near-singular pairs.  With P = s(ub) the
// point of the segment closest to the target (distance d) and b = d / |s'(ub)|
// the width of the integrand's peak in parameter units, the substitution
// u = ub + b sinh(mu) (the sinh transformation of nearly singular integrals)
// spreads the peak evenly over mu; each side of it, mu in [asinh(-ub/b), 0]
// and [0, asinh((1-ub)/b)], takes the 16-point Gauss-Legendre rule.  The
// same rule applied to the straight segment tangent to the curve at P
// (|P - s(0)| back, |s(1) - P| forward), whose integral is known in closed
// form, serves as a control variate: its exact integral minus its rule value
// is added, which removes most of the rule's error near the peak (the
// curve's integrand approaches the tangent's as d -> 0).  Every pair costs
// the same (32 + 32 kernel evaluations): no panel recursion, no divergence.
template <int DEG>
__device__ __forceinline__ void mapped_half_seg(const Seg &s, const double *xs, double ub,
                                                double b, double m0, double m1, const NsRule &R,
                                                double *acc) {
    const double hw = 0.5 * (m1 - m0), mc = 0.5 * (m1 + m0);
    if (!(hw > 0.0)) return;
    for (int k = 0; k < kNsGL; k++) {
        const double mu = mc + hw * R.x[k];
        const double e = exp(mu), ei = 1.0 / e;
        const double u = ub + b * 0.5 * (e - ei);
        const double jac = R.w[k] * hw * b * 0.5 * (e + ei);
        double r[3], d[3];
        for (int q = 0; q < 3; q++) {
            r[q] = seg_p<DEG>(s, q, u) - xs[q];
            d[q] = seg_d<DEG>(s, q, u);
        }
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double y = rsqrt_nr(r2);
        const double f = jac * (y * y * y);
        acc[0] += f * (r[1] * d[2] - r[2] * d[1]);
        acc[1] += f * (r[2] * d[0] - r[0] * d[2]);
        acc[2] += f * (r[0] * d[1] - r[1] * d[0]);
    }
}

// the rule on the straight segment P + l t, l in [-la, lb] (t unit), peak at
// l0 (its point closest to x) of width dd; acc -= rule, the caller adds the
// closed form
__device__ __forceinline__ void mapped_half_line(const double *rho, const double *t, double l0,
                                                 double dd, double m0, double m1,
                                                 const NsRule &R, double *acc) {
    const double hw = 0.5 * (m1 - m0), mc = 0.5 * (m1 + m0);
    if (!(hw > 0.0)) return;
    // (r x t) = (rho + l t) x t = rho x t for every l
    const double c[3] = {rho[1] * t[2] - rho[2] * t[1], rho[2] * t[0] - rho[0] * t[2],
                         rho[0] * t[1] - rho[1] * t[0]};
    const double rt = rho[0] * t[0] + rho[1] * t[1] + rho[2] * t[2];
    const double rr = rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2];
    double sum = 0.0;
    for (int k = 0; k < kNsGL; k++) {
        const double mu = mc + hw * R.x[k];
        const double e = exp(mu), ei = 1.0 / e;
        const double l = l0 + dd * 0.5 * (e - ei);
        const double jac = R.w[k] * hw * dd * 0.5 * (e + ei);
        const double r2 = rr + 2.0 * l * rt + l * l;
        const double y = rsqrt_nr(r2);
        sum += jac * (y * y * y);
    }
    acc[0] -= sum * c[0];
    acc[1] -= sum * c[1];
    acc[2] -= sum * c[2];
}

template <int DEG>
__device__ void ns_seg_mapped(const Seg &s, const double *xs, const NsRule &R, double *acc) {
    const double ub = closest_u<DEG>(s, xs);
    double P[3], d1[3], S0[3], S1[3], dummy[3];
    seg_eval<DEG>(s, ub, P, d1);
    seg_eval<DEG>(s, 0.0, S0, dummy);
    seg_eval<DEG>(s, 1.0, S1, dummy);
    double dist2 = 0.0, sp2 = 0.0, la = 0.0, lb = 0.0;
    for (int q = 0; q < 3; q++) {
        dist2 += (P[q] - xs[q]) * (P[q] - xs[q]);
        sp2 += d1[q] * d1[q];
        la += (P[q] - S0[q]) * (P[q] - S0[q]);
        lb += (S1[q] - P[q]) * (S1[q] - P[q]);
    }
    la = sqrt(la); lb = sqrt(lb);
    const double sn = sqrt(sp2);
    double b = sqrt(dist2) / sn;
    b = b < 1e-13 ? 1e-13 : b;
    acc[0] = acc[1] = acc[2] = 0.0;
    mapped_half_seg<DEG>(s, xs, ub, b, asinh(-ub / b), 0.0, R, acc);
    mapped_half_seg<DEG>(s, xs, ub, b, 0.0, asinh((1.0 - ub) / b), R, acc);
    // control variate: tangent segment at P
    double t[3], rho[3], A[3], B[3], cv[3];
    for (int q = 0; q < 3; q++) {
        t[q] = d1[q] / sn;
        rho[q] = P[q] - xs[q];
        A[q] = P[q] - la * t[q];
        B[q] = P[q] + lb * t[q];
    }
    chord_raw(A, B, xs, cv);
    double l0 = -(rho[0] * t[0] + rho[1] * t[1] + rho[2] * t[2]);
    l0 = l0 < -la ? -la : (l0 > lb ? lb : l0);
    double dd2 = 0.0;
    for (int q = 0; q < 3; q++) {
        const double v = rho[q] + l0 * t[q];
        dd2 += v * v;
    }
    double dd = sqrt(dd2);
    dd = dd < 1e-13 * (la + lb) ? 1e-13 * (la + lb) : dd;
    for (int q = 0; q < 3; q++) acc[q] += cv[q];
    mapped_half_line(rho, t, l0, dd, asinh((-la - l0) / dd), 0.0, R, acc);
    mapped_half_line(rho, t, l0, dd, 0.0, asinh((lb - l0) / dd), R, acc);
}

// mapped segment integral minus the Q-point sum, for one (node, segment) pair
template <int DEG>
__device__ void ns_pair_mapped(int o, int sg, int sh, const int *off, const int *fil,
                               const double *x, const double *xn, const double *D,
                               const double *S, const double *dtau, const double *gamma,
                               const double *qpos, const double *qchg, int Q, double L,
                               const NsRule &R, double *out) {
    double xs[3];
    unpack_shift(sh, x + 3 * o, L, xs);
    Seg s = load_seg(sg, off, fil, x, xn, D, S, dtau);
    double acc[3], qs[3];
    ns_seg_mapped<DEG>(s, xs, R, acc);
    ns_qsum(sg, xs, qpos, qchg, Q, qs);
    const double g4 = gamma[fil[sg]] / (4.0 * kPi);
    for (int q = 0; q < 3; q++) out[q] = g4 * acc[q] - qs[q] / (4.0 * kPi);
}

// every pair (list == nullptr, count = total pairs), or the pairs listed
__global__ __launch_bounds__(256) void k_ns_mapped(
    const int *__restrict__ count, const int *__restrict__ list, const int *__restrict__ pnode,
    const int2 *__restrict__ pairs, const int *__restrict__ off, const int *__restrict__ fil,
    const double *__restrict__ x, const double *__restrict__ xn, const double *__restrict__ D,
    const double *__restrict__ S, const double *__restrict__ dtau,
    const double *__restrict__ gamma, const double *__restrict__ qpos,
    const double *__restrict__ qchg, int Q, double L, NsRule R, double *__restrict__ pout) {
    const int n = *count;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int p = list ? list[i] : i;
        const int2 pr = pairs[p];
        double out[3];
        if (S)
            ns_pair_mapped<5>(pnode[p], pr.x, pr.y, off, fil, x, xn, D, S, dtau, gamma, qpos, qchg,
                              Q, L, R, out);
        else
            ns_pair_mapped<3>(pnode[p], pr.x, pr.y, off, fil, x, xn, D, S, dtau, gamma, qpos, qchg,
                              Q, L, R, out);
        pout[3 * (size_t)p] = out[0];
        pout[3 * (size_t)p + 1] = out[1];
        pout[3 * (size_t)p + 2] = out[2];
    }
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
        s.c4[q] = s.c5[q] = 0.0;
    }
    seg_derivs(s);
    double I[3];
    ns_seg_integral<3>(s, x, R, I);
    const TangentBase tb = tangent_baseline(s, x, 1.0);
    NsFrame F = ns_frame(A, B, D0, D1, x);
    for (int k = 0; k < 8; k++) X[8 * i + k] = F.f[k];
    for (int q = 0; q < 3; q++) T[3 * i + q] = (float)((I[q] - tb.I[q]) / tb.mult);
    if (aux) {
        double *o = aux + 7 * i;
        o[0] = tb.dstar;
        o[1] = I[0]; o[2] = I[1]; o[3] = I[2];
        o[4] = tb.mult;
        o[5] = tb.S;
        o[6] = F.dc;
    }
}

// Pair (target o, segment sg): end points, the end tangents ds/du of the
// segment over u in [0, 1] in units of its chord length h (the sample box's
// frame), and the image-shifted target.
__device__ __forceinline__ void pair_geometry(int o, int sg, int sh, const int *off, const int *fil,
                                              const double *x, const double *xn, const double *D,
                                              const double *dtau, double L, double *A,
                                              double *B, double *D0, double *D1, double *xs) {
    int jn = next_node_d(off, fil, sg);
    double h2 = 0.0;
    for (int q = 0; q < 3; q++) {
        A[q] = x[3 * sg + q]; B[q] = xn[3 * sg + q];
        h2 += (B[q] - A[q]) * (B[q] - A[q]);
    }
    const double sc = dtau[sg] / sqrt(h2);
    for (int q = 0; q < 3; q++) {
        D0[q] = sc * D[3 * sg + q];
        D1[q] = sc * D[3 * jn + q];
    }
    unpack_shift(sh, x + 3 * o, L, xs);
}

// Split the pairs by the error indicator before any inference: a pair whose
// inputs lie in the sample box and whose bin error fits the budget gets its
// features written at slot i of the learned list (learn[i] = pair), every
// other pair goes to the plain integrator's list; so the network runs only on the
// pairs it carries (lists in no particular order).
__global__ __launch_bounds__(256) void k_ns_select(
    const int *__restrict__ total, int N, const int *__restrict__ pnode,
    const int2 *__restrict__ pairs, const int *__restrict__ off, const int *__restrict__ fil,
    const double *__restrict__ x, const double *__restrict__ xn, const double *__restrict__ D,
    const double *__restrict__ dtau, const double *__restrict__ gamma, double L, NsBox box,
    const double *__restrict__ vscale, float *__restrict__ X, int *__restrict__ counts,
    int *__restrict__ learn, int *__restrict__ fb_list) {
    if (!counts[2]) return;   // the gate rules every pair out
    const int P = *total;
    // allowed rms error of one pair's raw integral times |Gamma| / (4 pi h)
    const double budget = box.tol * vscale[0] / sqrt((double)P / (double)(N > 0 ? N : 1));
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        int2 pr = pairs[p];
        double A[3], B[3], D0[3], D1[3], xs[3];
        pair_geometry(pnode[p], pr.x, pr.y, off, fil, x, xn, D, dtau, L, A, B, D0, D1, xs);
        NsFrame F = ns_frame(A, B, D0, D1, xs);
        const double g4 = gamma[fil[pr.x]] / (4.0 * kPi);
        const bool ok = F.inbox && (double)box.err[ns_bin(F.dc)] * fabs(g4) / F.h <= budget;
        if (ok) {
            const int i = atomicAdd(&counts[0], 1);
            learn[i] = p;
            for (int k = 0; k < 8; k++) X[8 * (size_t)i + k] = F.f[k];
        } else {
            fb_list[atomicAdd(&counts[1], 1)] = p;
        }
    }
}

// learned segment integral of the listed pairs: I_tan + mult * (network
// output in the chord frame), minus the Q-point sum the pair kernel added
__global__ __launch_bounds__(256) void k_ns_combine(
    const int *__restrict__ nlearn, const int *__restrict__ learn, const int *__restrict__ pnode,
    const int2 *__restrict__ pairs, const int *__restrict__ off, const int *__restrict__ fil,
    const double *__restrict__ x, const double *__restrict__ xn, const double *__restrict__ D,
    const double *__restrict__ dtau, const double *__restrict__ gamma,
    const double *__restrict__ qpos, const double *__restrict__ qchg, int Q, double L,
    const float *__restrict__ Y, double *__restrict__ pout) {
    const int n = *nlearn;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int p = learn[i];
        int2 pr = pairs[p];
        double A[3], B[3], D0[3], D1[3], xs[3];
        pair_geometry(pnode[p], pr.x, pr.y, off, fil, x, xn, D, dtau, L, A, B, D0, D1, xs);
        NsFrame F = ns_frame(A, B, D0, D1, xs);
        const double g4 = gamma[fil[pr.x]] / (4.0 * kPi);
        Seg sgm = load_seg(pr.x, off, fil, x, xn, D, nullptr, dtau);
        const TangentBase tb = tangent_baseline(sgm, xs, F.h);
        double qs[3], y[3];
        for (int k = 0; k < 3; k++) y[k] = (double)Y[3 * (size_t)i + k] * tb.mult;
        ns_qsum(pr.x, xs, qpos, qchg, Q, qs);
        for (int q = 0; q < 3; q++) {
            double yw = F.e[0][q] * y[0] + F.e[1][q] * y[1] + F.e[2][q] * y[2];
            pout[3 * (size_t)p + q] = g4 * (tb.I[q] + yw) - qs[q] / (4.0 * kPi);
        }
    }
}

// The velocity scale v_scale = rms over the nodes of |base_i|, and a bound
// that decides for all pairs at once whether the network can take any: with
// e_min the table's smallest entry, h_max the longest chord and G the
// smallest |Gamma|, every pair's indicator is at least e_min G / (4 pi h_max)
// sqrt(P / N), so none passes when that exceeds tol v_scale.  Then the
// selection and the inference do nothing and the plain integrator takes
// every pair in pair order.  Two passes, fixed order: per block sums of
// squares, longest chord and smallest |Gamma|, then one block that forms the
// scale and the decision (gate[0] = 1: some pair may pass; gate[1] =
// !gate[0]).
constexpr int kNsVsBlocks = 256;
__global__ __launch_bounds__(256) void k_ns_gate_part(int N, const double *__restrict__ base,
                                                      const double *__restrict__ x,
                                                      const double *__restrict__ xn,
                                                      const int *__restrict__ fil,
                                                      const double *__restrict__ gamma,
                                                      double *__restrict__ part) {
    __shared__ double s2[256], sh[256], sg[256];
    double a = 0.0, hm = 0.0, gm = INFINITY;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        double c2 = 0.0;
        for (int q = 0; q < 3; q++) {
            a += base[3 * i + q] * base[3 * i + q];
            const double d = xn[3 * i + q] - x[3 * i + q];
            c2 += d * d;
        }
        hm = fmax(hm, c2);
        gm = fmin(gm, fabs(gamma[fil[i]]));
    }
    s2[threadIdx.x] = a;
    sh[threadIdx.x] = hm;
    sg[threadIdx.x] = gm;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s2[threadIdx.x] += s2[threadIdx.x + o];
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
            sg[threadIdx.x] = fmin(sg[threadIdx.x], sg[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = s2[0];
        part[3 * blockIdx.x + 1] = sh[0];
        part[3 * blockIdx.x + 2] = sg[0];
    }
}
__global__ __launch_bounds__(256) void k_ns_gate_final(int N, const double *__restrict__ part,
                                                       int nparts, const int *__restrict__ total,
                                                       double emin, double tol,
                                                       double *__restrict__ vscale,
                                                       int *__restrict__ gate) {
    __shared__ double s2[256], sh[256], sg[256];
    double a = 0.0, hm = 0.0, gm = INFINITY;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        a += part[3 * i];
        hm = fmax(hm, part[3 * i + 1]);
        gm = fmin(gm, part[3 * i + 2]);
    }
    s2[threadIdx.x] = a;
    sh[threadIdx.x] = hm;
    sg[threadIdx.x] = gm;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s2[threadIdx.x] += s2[threadIdx.x + o];
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
            sg[threadIdx.x] = fmin(sg[threadIdx.x], sg[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double vs = N > 0 ? sqrt(s2[0] / N) : 0.0;
        const double P = (double)*total;
        const double hmax = sqrt(sh[0]);
        const bool some = P > 0.0 && hmax > 0.0 &&
                          emin * sg[0] / (4.0 * kPi * hmax) * sqrt(P / (double)N) <= tol * vs;
        vscale[0] = vs;
        gate[0] = some ? 1 : 0;
        gate[1] = some ? 0 : 1;
    }
}

// flag + list build (after geometry and binning)
void ns_build_pairs(bs_plan_t p) {
    const int N = (int)p->N, bs = 256;
    const int nb3 = p->ns_ncmax * p->ns_ncmax * p->ns_ncmax;
    int *ncp = (int *)p->ns_nc.p;
    int *ckey = (int *)p->ns_ckey.p, *ccnt = (int *)p->ns_ccnt.p, *cstart = (int *)p->ns_cstart.p;
    int *cfill = (int *)p->ns_cfill.p, *cperm = (int *)p->ns_cperm.p;
    const int *off = (const int *)p->d_off.p, *fil = (const int *)p->d_fil.p;
    const double *x = (const double *)p->d_x.p, *ell = (const double *)p->d_ell.p;
    const double *xn = (const double *)p->d_xn.p;
    double *red = (double *)p->ns_red.p;
    const int nred = ceil_div(N, bs) < kNsRedBlocks ? ceil_div(N, bs) : kNsRedBlocks;
    hipLaunchKernelGGL(k_ns_reach, dim3(nred), dim3(bs), 0, p->stream, N, x, xn, ell,
                       p->prm.ns_eta, red + 1, red + 1 + kNsRedBlocks);
    hipLaunchKernelGGL(k_ns_cells, dim3(1), dim3(bs), 0, p->stream, red + 1,
                       red + 1 + kNsRedBlocks, nred, N, p->prm.L, p->ns_ncmax, red, ncp);
    int *tkey = (int *)p->ns_tkey.p, *tcnt = (int *)p->ns_tcnt.p, *tstart = (int *)p->ns_tstart.p;
    int *tfill = (int *)p->ns_tfill.p, *tperm = (int *)p->ns_tperm.p;
    // segment keys span both grids (nc_B <= nc_A <= ncmax)
    hipLaunchKernelGGL(k_ns_zero, dim3(ceil_div(2 * nb3 + 1, bs)), dim3(bs), 0, p->stream,
                       2 * nb3 + 1, ccnt, cfill);
    hipLaunchKernelGGL(k_ns_zero, dim3(ceil_div(nb3 + 1, bs)), dim3(bs), 0, p->stream, nb3 + 1,
                       tcnt, tfill);
    hipLaunchKernelGGL(k_ns_keys, dim3(ceil_div(N, bs)), dim3(bs), 0, p->stream, N, x, xn,
                       ell, p->prm.ns_eta, p->prm.L, (const int *)ncp, ckey, ccnt, tkey, tcnt);
    int *sums = (int *)p->scan_tmp.p;   // the search may run on the side stream
    exclusive_scan(p, ccnt, cstart, 2 * nb3, sums);
    exclusive_scan(p, tcnt, tstart, nb3, sums);
    hipLaunchKernelGGL(k_ns_scatter, dim3(ceil_div(N, bs)), dim3(bs), 0, p->stream, N,
                       (const int *)ckey, (const int *)cstart, cfill, cperm, (const int *)tkey,
                       (const int *)tstart, tfill, tperm);
    const int nsort = 2 * nb3 < 4096 ? 2 * nb3 : 4096;
    hipLaunchKernelGGL(k_ns_sort, dim3(nsort), dim3(64), 0, p->stream, (const int *)ncp,
                       (const int *)cstart, cperm, ckey);
    hipLaunchKernelGGL(k_ns_gather, dim3(ceil_div(N, bs)), dim3(bs), 0, p->stream, N,
                       (const int *)cperm, x, xn, ell, p->prm.ns_eta, p->prm.L,
                       (double4 *)p->ns_segA.p, (double4 *)p->ns_segB.p,
                       (float4 *)p->ns_segM.p, (float4 *)p->ns_segH.p);
    NsArgs a;
    a.N = N; a.max_per_node = p->ns_max_per_node;
    a.L = p->prm.L; a.eta = p->prm.ns_eta;
    a.x = x; a.off = off; a.fil = fil;
    a.ncp = ncp; a.cstart = cstart;
    a.segA = (const double4 *)p->ns_segA.p; a.segB = (const double4 *)p->ns_segB.p;
    a.segM = (const float4 *)p->ns_segM.p; a.segH = (const float4 *)p->ns_segH.p;
    a.segj = (const int *)cperm;
    int *cnt = (int *)p->ns_cnt.p, *start = (int *)p->ns_start.p;
    // exactly one of the two does work, depending on the cell count.  The
    // cells' target counts are uneven, so the cell kernel's workgroups stride
    // over many more cells than fit at once (~1500 resident): 20000 of them
    // balance the last rounds better than 8192 (1.58 -> 1.53 ms on the
    // 1e6-node tangle), while one per cell pays for the many empty ones.
    constexpr int kNsFlagBlocks = 20000;
    hipLaunchKernelGGL(k_ns_flag_cells, dim3(nb3 < kNsFlagBlocks ? nb3 : kNsFlagBlocks), dim3(bs), 0, p->stream, a,
                       (const int *)tstart, (const int *)tperm, cnt, (int2 *)p->ns_slots.p,
                       (int *)p->d_status.p);
    const int nwave = ceil_div((int64_t)N * 64, bs);
    hipLaunchKernelGGL(k_ns_flag, dim3(nwave < 1024 ? nwave : 1024), dim3(bs), 0, p->stream, a,
                       cnt, (int2 *)p->ns_slots.p, (int *)p->d_status.p);
    exclusive_scan(p, cnt, start, N, sums);
    hipLaunchKernelGGL(k_ns_compact, dim3(ceil_div((int64_t)N * kNsCompactLanes, bs)), dim3(bs),
                       0, p->stream, N, p->ns_max_per_node, (const int *)cnt, (const int *)start,
                       (const int2 *)p->ns_slots.p, (int2 *)p->ns_pairs.p, (int *)p->ns_pnode.p);
}

void ns_rule(NsRule *R);

// the graded-panel integrator on every pair (list == nullptr) or on the
// listed ones; nothing when *skip is set.  The pair count is known on the
// device only: the grid strides over it with many more workgroups than fit
// at once (1024 resident at four wavefronts per SIMD), so that the last
// round does not leave most CUs idle (1024 workgroups: 1.48 ms for the
// 1.1e7 pairs of the 1e6-node tangle at three wavefronts per SIMD; 12288:
// 1.36 ms)
constexpr int kNsIntegrateBlocks = 12288;

static void adaptive_pairs(bs_plan_t p, const int *count, const int *list,
                           const int *skip = nullptr) {
    NsRule R;
    ns_rule(&R);
    hipLaunchKernelGGL(k_ns_integrate, dim3(kNsIntegrateBlocks), dim3(256), 0, p->stream,
                       count, list, (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_xn.p,
                       (const double *)p->d_D.p, p->order == 6 ? (const double *)p->d_sdd.p : nullptr,
                       (const double *)p->d_dtau.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_qpos.p, (const double *)p->d_qchg.p, p->Q,
                       p->prm.L, R, (double *)p->ns_pout.p, skip);
}

void launch_ns_adaptive(bs_plan_t p, double *v) {
    const int N = (int)p->N;
    const int *start = (const int *)p->ns_start.p;
    adaptive_pairs(p, start + N, nullptr);
    hipLaunchKernelGGL(k_ns_apply, dim3(ceil_div(N, 256)), dim3(256), 0, p->stream, N, start,
                       (const double *)p->ns_pout.p, v);
}

// the mapped rule on every pair (list == nullptr) or on the listed ones
static void mapped_pairs(bs_plan_t p, const int *count, const int *list) {
    NsRule R;
    ns_rule(&R);
    hipLaunchKernelGGL(k_ns_mapped, dim3(2048), dim3(256), 0, p->stream, count, list,
                       (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_xn.p,
                       (const double *)p->d_D.p, p->order == 6 ? (const double *)p->d_sdd.p : nullptr,
                       (const double *)p->d_dtau.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_qpos.p, (const double *)p->d_qchg.p, p->Q,
                       p->prm.L, R, (double *)p->ns_pout.p);
}

void launch_ns_mapped(bs_plan_t p, double *v) {
    const int N = (int)p->N;
    const int *start = (const int *)p->ns_start.p;
    mapped_pairs(p, start + N, nullptr);
    hipLaunchKernelGGL(k_ns_apply, dim3(ceil_div(N, 256)), dim3(256), 0, p->stream, N, start,
                       (const double *)p->ns_pout.p, v);
}

void launch_ns_mlp(bs_plan_t p, double *v, const double *base) {
    const int N = (int)p->N;
    const int *start = (const int *)p->ns_start.p;
    const int *total = start + N;
    NsBox box;
    double emin = INFINITY;
    for (int b = 0; b < kNsBins; b++) {
        box.err[b] = p->ns_err[b];
        emin = std::min(emin, (double)p->ns_err[b]);
    }
    box.tol = p->prm.tol;
    // cnt: [0] learned pairs, [1] listed plain-integrator pairs, [2] gate, [3] !gate
    int *cnt = (int *)p->ns_fallback.p;
    int *learn = (int *)p->ns_learn.p;
    double *vs = (double *)p->ns_vs.p;   // [0] v_scale, [1..] per-block partials
    const int nvs = std::min(kNsVsBlocks, std::max(1, ceil_div((int64_t)N, 256)));
    hipLaunchKernelGGL(k_ns_zero, dim3(1), dim3(64), 0, p->stream, 1, cnt, cnt + 1);
    hipLaunchKernelGGL(k_ns_gate_part, dim3(nvs), dim3(256), 0, p->stream, N, base,
                       (const double *)p->d_x.p, (const double *)p->d_xn.p,
                       (const int *)p->d_fil.p, (const double *)p->d_gamma.p, vs + 1);
    hipLaunchKernelGGL(k_ns_gate_final, dim3(1), dim3(256), 0, p->stream, N,
                       (const double *)(vs + 1), nvs, total, emin, p->prm.tol, vs, cnt + 2);
    hipLaunchKernelGGL(k_ns_select, dim3(1024), dim3(256), 0, p->stream, total, N,
                       (const int *)p->ns_pnode.p, (const int2 *)p->ns_pairs.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_x.p, (const double *)p->d_xn.p,
                       (const double *)p->d_D.p, (const double *)p->d_dtau.p,
                       (const double *)p->d_gamma.p, p->prm.L, box, (const double *)vs,
                       (float *)p->ns_X.p, cnt, learn, (int *)p->ns_fblist.p);
    mlp_forward_device(p->mlp, cnt, (int64_t)N * p->ns_max_per_node, (const float *)p->ns_X.p,
                       (float *)p->ns_Y.p, p->stream);
    hipLaunchKernelGGL(k_ns_combine, dim3(1024), dim3(256), 0, p->stream, (const int *)cnt,
                       (const int *)learn, (const int *)p->ns_pnode.p,
                       (const int2 *)p->ns_pairs.p, (const int *)p->d_off.p,
                       (const int *)p->d_fil.p, (const double *)p->d_x.p,
                       (const double *)p->d_xn.p, (const double *)p->d_D.p,
                       (const double *)p->d_dtau.p, (const double *)p->d_gamma.p,
                       (const double *)p->d_qpos.p, (const double *)p->d_qchg.p, p->Q, p->prm.L,
                       (const float *)p->ns_Y.p, (double *)p->ns_pout.p);
    // the refused pairs (gate open), or every pair in order (gate closed)
    adaptive_pairs(p, cnt + 1, (const int *)p->ns_fblist.p, cnt + 3);
    adaptive_pairs(p, total, nullptr, cnt + 2);
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

// ------------------------------------------------------ learned error table
namespace bs {

// per-block sums of squared errors, counts and maxima per bin: the error of
// one sample is |I_learned - I| = mult |y - t| (raw integral, h = 1), binned
// by its distance to the chord over h
__global__ __launch_bounds__(256) void k_ns_err_part(int64_t n, const float *__restrict__ Y,
                                                     const float *__restrict__ T,
                                                     const double *__restrict__ aux,
                                                     double *__restrict__ part) {
    double e2[kNsBins], cnt[kNsBins], mx[kNsBins];
#pragma unroll
    for (int b = 0; b < kNsBins; b++) e2[b] = cnt[b] = mx[b] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < 3; k++) {
            const double d = (double)Y[3 * i + k] - (double)T[3 * i + k];
            s += d * d;
        }
        const double e = aux[7 * i + 4] * sqrt(s);
        const int bin = ns_bin(aux[7 * i + 6]);
#pragma unroll
        for (int b = 0; b < kNsBins; b++) {
            const bool m = b == bin;
            e2[b] += m ? e * e : 0.0;
            cnt[b] += m ? 1.0 : 0.0;
            mx[b] = m ? fmax(mx[b], e) : mx[b];
        }
    }
    __shared__ double sh[256];
    double *out = part + (size_t)blockIdx.x * kNsBins * 3;
    for (int b = 0; b < kNsBins; b++) {
        for (int w = 0; w < 3; w++) {
            double v = 0.0;
#pragma unroll
            for (int bb = 0; bb < kNsBins; bb++)
                if (bb == b) v = w == 0 ? e2[bb] : (w == 1 ? cnt[bb] : mx[bb]);
            sh[threadIdx.x] = v;
            __syncthreads();
            for (int o = blockDim.x / 2; o > 0; o >>= 1) {
                if (threadIdx.x < o)
                    sh[threadIdx.x] = w == 2 ? fmax(sh[threadIdx.x], sh[threadIdx.x + o])
                                             : sh[threadIdx.x] + sh[threadIdx.x + o];
                __syncthreads();
            }
            if (threadIdx.x == 0) out[3 * b + w] = sh[0];
            __syncthreads();
        }
    }
}

// rms and max per bin over the blocks, in block order; +inf where a bin
// holds no sample (the network is never used there)
__global__ void k_ns_err_final(int nparts, const double *__restrict__ part,
                               float *__restrict__ rms, float *__restrict__ mx) {
    const int b = threadIdx.x;
    if (b >= kNsBins) return;
    double e2 = 0.0, c = 0.0, m = 0.0;
    for (int k = 0; k < nparts; k++) {
        const double *q = part + ((size_t)k * kNsBins + b) * 3;
        e2 += q[0];
        c += q[1];
        m = fmax(m, q[2]);
    }
    if (rms) rms[b] = c > 0.0 ? (float)sqrt(e2 / c) : INFINITY;
    if (mx) mx[b] = c > 0.0 ? (float)m : INFINITY;
}

constexpr int kNsErrBlocks = 256;

// Y: inference output scratch [n][3]; part: [kNsErrBlocks][bins][3];
// table: [2][bins] device
int ns_error_table(bs_mlp_t m, int64_t n, const float *X, const float *T, const double *aux,
                   float *Y, double *part, float *table, float *rms_out, float *max_out) {
    hipStream_t st = mlp_stream(m);
    int rc = bs_mlp_forward(m, n, X, Y);
    if (rc) return rc;
    const int nb = (int)std::min<int64_t>(kNsErrBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_ns_err_part, dim3(nb), dim3(256), 0, st, n, Y, T, aux, part);
    hipLaunchKernelGGL(k_ns_err_final, dim3(1), dim3(64), 0, st, nb, (const double *)part, table,
                       table + kNsBins);
    float host[2 * kNsBins];
    if (hipMemcpyAsync(host, table, sizeof(host), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return BS_EDEVICE;
    for (int b = 0; b < kNsBins; b++) {
        if (rms_out) rms_out[b] = host[b];
        if (max_out) max_out[b] = host[kNsBins + b];
    }
    return BS_OK;
}

}  // namespace bs

// ------------------------------------------- error table without allocation
// Callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid it) use a file-scope device array for
// the network outputs, the per-block partial sums and the table.  Each GPU
// holds its own copy for the life of the process; host code reaches it only
// through the device address taken once per device by hipGetSymbolAddress
// (the array's name is a host-side stand-in).  Calls on one GPU share it:
// calls that overlap on one GPU race.
namespace bs {
constexpr int64_t kNsErrNoAllocMax = 1 << 18;   // samples per call, at most
constexpr size_t kNsScratchY = sizeof(float) * 3 * (size_t)kNsErrNoAllocMax;
constexpr size_t kNsScratchPart = sizeof(double) * 3 * kNsBins * kNsErrBlocks;
constexpr size_t kNsScratchBytes = kNsScratchY + kNsScratchPart + 256;
static __device__ __align__(256) unsigned char scratch[kNsScratchBytes];

constexpr int kNsMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kNsMaxDevices];

// device address of this device's scratch (taken on the first call on it)
static int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNsMaxDevices) return BS_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return BS_EDEVICE;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return BS_OK;
}
}  // namespace bs

extern "C" int bs_ns_error_table_noalloc(bs_mlp_t m, int64_t n, const float *X, const float *T,
                                         const double *aux, float *rms_out, float *max_out,
                                         int nbins) {
    if (!m || n < 1 || !X || !T || !aux || nbins != bs::kNsBins) return BS_EINVAL;
    if (n > bs::kNsErrNoAllocMax) return BS_EINVAL;   // beyond the static scratch
    void *base = nullptr;
    int rc = bs::scratch_address(&base);
    if (rc) return rc;
    unsigned char *sp = (unsigned char *)base;
    float *Y = (float *)sp;
    double *part = (double *)(sp + bs::kNsScratchY);
    hipStream_t st = bs::mlp_stream(m);
    if ((rc = bs_mlp_forward(m, n, X, Y))) return rc;
    const int nb = (int)std::min<int64_t>(bs::kNsErrBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(bs::k_ns_err_part, dim3(nb), dim3(256), 0, st, n, Y, T, aux, part);
    hipLaunchKernelGGL(bs::k_ns_err_final, dim3(1), dim3(64), 0, st, nb, (const double *)part,
                       rms_out, max_out);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

extern "C" int bs_ns_error_table(bs_mlp_t m, int64_t n, const float *X, const float *T,
                                 const double *aux, float *rms_out, float *max_out, int nbins) {
    if (!m || n < 1 || !X || !T || !aux || nbins != bs::kNsBins) return BS_EINVAL;
    float *Y = nullptr, *table = nullptr;
    double *part = nullptr;
    if (hipMalloc((void **)&Y, sizeof(float) * 3 * (size_t)n) != hipSuccess ||
        hipMalloc((void **)&part, sizeof(double) * 3 * bs::kNsBins * bs::kNsErrBlocks) !=
            hipSuccess ||
        hipMalloc((void **)&table, sizeof(float) * 2 * bs::kNsBins) != hipSuccess) {
        (void)hipFree(Y); (void)hipFree(part); (void)hipFree(table);
        return BS_ENOMEM;
    }
    int rc = bs::ns_error_table(m, n, X, T, aux, Y, part, table, rms_out, max_out);
    (void)hipStreamSynchronize(bs::mlp_stream(m));
    (void)hipFree(Y); (void)hipFree(part); (void)hipFree(table);
    return rc;
}
