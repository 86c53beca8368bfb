// Short-range part (Sec. 3.2, eq:velocity_shortrange and
// eq:streamfunction_shortrange) as quadrature sums over cell lists, and the
// energy reduction (eq:kinetic_energy_streamfunction).
//
// A wavefront per target node, nodes processed in cell order so that
// consecutive wavefronts read the same few cells.  For each quadrature point
// of the 4 x 4 x 4 cells (edge >= 2 r_c / 3) from the cell of x - r_c on (or
// of every cell when fewer than 4 fit along an axis):
// r = s_q - s_i by minimum image (formed in float64), skip the 2Q points of
// the two segments adjacent to the node, keep r < r_c, and add
//   v:   g_sr(r) (r x q) / r^3,  g_sr = erfc(alpha r) + (2 alpha r/sqrt(pi)) e^{-alpha^2 r^2}
//   psi: erfc(alpha r) q / r
// times 1/(4 pi).  R = float in the mixed mode (float32 accumulation).
#include "bs_internal.h"
#include "bs_device.h"
#include "erfcx_fit.h"

namespace bs {

// g_sr(x) = erfc(x) + (2/sqrt(pi)) x exp(-x^2) = exp(-x^2) (erfcx(x) +
// (2/sqrt(pi)) x): one exponential, with erfcx = P(Z) / (4 + x),
// Z = (4 - x) / (4 + x), from its fitted polynomial (float64: relative
// error 3e-15 for x = alpha r below the beta of every tolerance in Table 1,
// 7e-14 where the term is below 1e-15 of its value at r = 0; float32:
// 4e-7, below the float32 rounding of exp(-x^2) for x near beta)
__device__ __forceinline__ double g_short(double x) {
    constexpr double two_over_sqrtpi = 1.12837916709551257389615890312154517;
    const double inv = 1.0 / (kErfcxShift + x);
    const double z = (kErfcxShift - x) * inv;
    double p = kErfcxP[kErfcxDeg];
#pragma unroll
    for (int k = kErfcxDeg - 1; k >= 0; k--) p = fma(p, z, kErfcxP[k]);
    return exp(-x * x) * fma(p, inv, two_over_sqrtpi * x);
}
__device__ __forceinline__ float g_short(float x) {
    constexpr float two_over_sqrtpi = 1.12837916709551257389615890312154517f;
    const float inv = __builtin_amdgcn_rcpf((float)kErfcxShift + x);
    const float z = ((float)kErfcxShift - x) * inv;
    float p = kErfcxP32[kErfcxDeg32];
#pragma unroll
    for (int k = kErfcxDeg32 - 1; k >= 0; k--) p = fmaf(p, z, kErfcxP32[k]);
    return expf(-x * x) * fmaf(p, inv, two_over_sqrtpi * x);
}

// One wavefront (four on small inputs) per target node.  Each lane holds one of the
// 4 x 4 x 4 cells around the target; the cells' contents are enumerated as one
// flattened range, 64 candidates per step (every lane busy, independent
// loads).  Only about a fifth of the candidates lie within r_c; in float64
// their separations are queued in LDS and their erfc / exp terms evaluated
// 64 at a time, so that the costly part runs with every lane busy (the
// float64 kernel was bound by those terms run for a whole wavefront per
// step: 3.5 -> 2.9 ms at 1e6 nodes).  The range is mapped to point indices
// in chunks of kMapCap: every
// lane writes its cell's run of point indices into the wavefront's own LDS
// map, and each candidate then takes its point index with one LDS read.  The
// partial sums are combined by a fixed xor-shuffle tree (deterministic order).
constexpr int kMapCap = 1024;
// accepted candidates queued per wavefront (a ring of two steps' worth)
constexpr int kQueue = 128;

template <typename R, bool PSI, int WPN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs(
    int N, int nc, int per_xcd, double L, double rc, double alpha,
                                               const int *__restrict__ nperm,
                                               const double *__restrict__ x,
                                               const int *__restrict__ off,
                                               const int *__restrict__ fil,
                                               const int *__restrict__ cstart,
                                               const double4 *__restrict__ spos,
                                               const R *__restrict__ schg,
                                               const double *__restrict__ base,
                                               double *__restrict__ out) {
    static_assert(WPN == 1 || WPN == 4, "1 or 4 wavefronts per target");
    __shared__ R red[4][3];
    __shared__ int pmap[4][kMapCap];
    // float64 only: in float32 the terms are cheap enough that the queue's
    // LDS round trips cost more than the idle lanes (measured slower)
    constexpr bool kQueued = sizeof(R) == 8;
    __shared__ R qbuf[kQueued ? 4 : 1][3][kQueued ? kQueue : 1];
    __shared__ int qpid[kQueued ? 4 : 1][kQueued ? kQueue : 1];
    const unsigned long long below = ((threadIdx.x & 63) == 0) ? 0ull
                                                               : (~0ull >> (64 - (threadIdx.x & 63)));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // WPN = 1: four targets per workgroup; WPN = 4: one target, its
    // candidate chunks dealt round-robin to the four wavefronts.  Targets
    // come in cell order, and consecutive workgroups of them stay on one XCD
    // (blocks b, b + 8, ... run on one XCD), so that the candidate windows
    // that neighbouring cells share are fetched into one L2
    const int blk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int t = WPN == 1 ? blk * 4 + wave : blk;
    const int part = WPN == 1 ? 0 : wave;
    if (t >= N) return;   // whole wavefronts (WPN = 1) or the whole workgroup
    const int o = nperm[t];
    const int ip = prev_node_d(off, fil, o);
    const double xi0 = x[3 * o], xi1 = x[3 * o + 1], xi2 = x[3 * o + 2];
    const double invL = 1.0 / L;
    // lanes 0..63: the 4 x 4 x 4 cells from the cell of x - r_c on (cells of
    // edge h >= 2 r_c / 3 hold every point within r_c in 4 per axis); a cell
    // whose box lies farther than r_c from x holds no partner and is dropped
    const int ncell = nc >= 4 ? 64 : 1;
    int cs = 0, cn = 0;
    if (lane < ncell) {
        int cidx = 0;
        bool near = true;
        if (nc >= 4) {
            const double ws[3] = {wrap_box(xi0, L), wrap_box(xi1, L), wrap_box(xi2, L)};
            const int dd[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
            const double h = L / nc;
            int c[3];
            double d2 = 0.0;
            for (int q = 0; q < 3; q++) {
                int v = (int)floor((ws[q] - rc) * invL * nc) + dd[q];
                // distance from x to the cell's extent [v h, (v + 1) h) (unwrapped)
                const double lo = v * h - ws[q], hi = ws[q] - (v + 1) * h;
                const double d = lo > 0.0 ? lo : (hi > 0.0 ? hi : 0.0);
                d2 += d * d;
                v %= nc;
                c[q] = v < 0 ? v + nc : v;
            }
            cidx = (c[2] * nc + c[1]) * nc + c[0];
            near = d2 <= rc * rc * (1.0 + 1e-12);
        }
        if (near) {
            cs = cstart[cidx];
            cn = cstart[cidx + 1] - cs;
        }
    }
    int incl = cn;
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, 63);
    const int excl = incl - cn;
    const R rc2 = (R)(rc * rc), a = (R)alpha;
    R acc0 = 0, acc1 = 0, acc2 = 0;
    static_assert(kMapCap % (64 * WPN) == 0, "chunks keep the lanes' candidate order");
    int *map = pmap[wave];
    R *qx = qbuf[kQueued ? wave : 0][0], *qy = qbuf[kQueued ? wave : 0][1],
      *qz = qbuf[kQueued ? wave : 0][2];
    int *qp = qpid[kQueued ? wave : 0];
    const int cs0 = __shfl(cs, 0);   // one cell (nc < 4): point index = cs0 + q
    // the kernel term of one candidate within r_c, separation f
    auto term = [&](R fx, R fy, R fz, int p) {
        const R r2 = fx * fx + fy * fy + fz * fz;
        const R rr = sqrt(r2);
        const R ar = a * rr;
        const R *qq = schg + 4 * (size_t)p;
        const R q0v = qq[0], q1v = qq[1], q2v = qq[2];
        if (PSI) {
            const R f = erfc(ar) / rr;
            acc0 += f * q0v; acc1 += f * q1v; acc2 += f * q2v;
        } else {
            const R g = g_short(ar);
            const R f = g / (r2 * rr);
            acc0 += f * (fy * q2v - fz * q1v);
            acc1 += f * (fz * q0v - fx * q2v);
            acc2 += f * (fx * q1v - fy * q0v);
        }
    };
    // separation of a candidate point (position and segment index sp): the
    // minimum-image separation (float64, then in R) and whether it lies
    // within r_c (the node's two adjacent segments excluded)
    auto sep = [&](const double4 &sp, R &fx, R &fy, R &fz) {
        const int sg = (int)sp.w;
        if (sg == o || sg == ip) return false;
        double rx = sp.x - xi0, ry = sp.y - xi1, rz = sp.z - xi2;
        rx -= L * rint(rx * invL);
        ry -= L * rint(ry * invL);
        rz -= L * rint(rz * invL);
        fx = (R)rx; fy = (R)ry; fz = (R)rz;
        const R r2 = fx * fx + fy * fy + fz * fz;
        return r2 < rc2 && r2 != (R)0;
    };
    // float64: ring of accepted candidates, positions [head, tail)
    // (wavefront-uniform); the terms of n <= 64 queued ones, one per lane
    int head = 0, tail = 0;
    auto drain = [&](int n) {
        if (lane < n) {
            const int sl = (head + lane) & (kQueue - 1);
            term(qx[sl], qy[sl], qz[sl], qp[sl]);
        }
        head += n;
    };
    // U steps of 64 candidates per round: their point indices, then all
    // their position loads, issued before any is used; the steps keep the
    // candidate order.  U = 1: the loads of a step ahead of its tests already
    // took the float64 kernel from 2.97 to 2.69 ms at 1e6 nodes; two steps
    // spill in float64 (and at three waves per SIMD ran slower), and in
    // float32 gained 4 % but changed the kernel's rounding (rel. error on the
    // ring pairs 1.03e-7 -> 1.54e-7), so they are not taken
    constexpr int U = 1;
    // chunks start at multiples of kMapCap (a multiple of 64 WPN), so every
    // wavefront meets its candidates in the same order as in one flat range
    for (int c0 = 0; c0 < total; c0 += kMapCap) {
        const int cend = min(total, c0 + kMapCap);
        if (ncell > 1) {
            const int lo = max(excl, c0), hi = min(excl + cn, cend);
            for (int j = lo; j < hi; j++) map[j - c0] = cs + (j - excl);
            wave_lds_sync();
        }
        for (int qb = c0 + part * 64; qb < cend; qb += 64 * WPN * U) {
            int pv[U];
            bool in[U];
            double4 sv[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = qb + u * 64 * WPN + lane;
                in[u] = q < cend;
                pv[u] = in[u] ? (ncell > 1 ? map[q - c0] : cs0 + q) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; u++) sv[u] = in[u] ? spos[pv[u]] : make_double4(0, 0, 0, -1);
#pragma unroll
            for (int u = 0; u < U; u++) {
                R fx = 0, fy = 0, fz = 0;
                const bool ok = in[u] && sep(sv[u], fx, fy, fz);
                if constexpr (kQueued) {
                    // the accepted ones (about a fifth) are queued in
                    // candidate order, and their erfc / exp terms run 64 at a
                    // time with every lane busy
                    const unsigned long long m = __ballot(ok);
                    if (ok) {
                        const int sl = (tail + __popcll(m & below)) & (kQueue - 1);
                        qx[sl] = fx; qy[sl] = fy; qz[sl] = fz; qp[sl] = pv[u];
                    }
                    tail += __popcll(m);
                    wave_lds_sync();
                    if (tail - head >= 64) {
                        drain(64);
                        wave_lds_sync();   // slots read before the next step writes them
                    }
                } else {
                    if (ok) term(fx, fy, fz, pv[u]);
                }
            }
        }
        if (ncell > 1) wave_lds_sync();   // map reads done before the next chunk is written
    }
    if constexpr (kQueued) drain(tail - head);   // fewer than 64 left
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        acc0 += __shfl_xor(acc0, m, 64);
        acc1 += __shfl_xor(acc1, m, 64);
        acc2 += __shfl_xor(acc2, m, 64);
    }
    if (WPN > 1) {
        if (lane == 0) { red[wave][0] = acc0; red[wave][1] = acc1; red[wave][2] = acc2; }
        __syncthreads();
        if (wave != 0) return;
        acc0 = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
        acc1 = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
        acc2 = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
    }
    if (lane == 0) {
        const double inv4pi = 1.0 / (4.0 * kPi);
        const double *b = base ? base : out;
        const double b0 = b[3 * o], b1 = b[3 * o + 1], b2 = b[3 * o + 2];
        out[3 * o] = b0 + (double)acc0 * inv4pi;
        out[3 * o + 1] = b1 + (double)acc1 * inv4pi;
        out[3 * o + 2] = b2 + (double)acc2 * inv4pi;
    }
}

// targets below this count get four wavefronts each (latency hiding on
// small inputs), but only when the pair sum runs alone: in the velocity,
// beside the spread and the transforms, one wavefront per target leaves them
// more of the chip (64^3 ellipses: 110 -> 107 us per evaluation)
constexpr int kPairSplitNodes = 16384;

template <typename R, bool PSI>
static void pairs_r(bs_plan_t p, const double *base, double *out, bool alone) {
    const int N = (int)p->N;
    const bool split = N < kPairSplitNodes && alone;
    const int nblk = split ? N : ceil_div(N, 4), per = ceil_div(nblk, 8);
    dim3 grid(8 * per), block(256);
    const double L = p->prm.L, rc = p->prm.rcut, alpha = p->prm.alpha;
    const int *nperm = (const int *)p->nd_perm.p, *off = (const int *)p->d_off.p,
              *fil = (const int *)p->d_fil.p, *cs = (const int *)p->pq_start.p;
    const double *x = (const double *)p->d_x.p;
    const double4 *sp = (const double4 *)p->pq_pos.p;
    const R *q = (const R *)p->pq_chg.p;
    if (split)
        hipLaunchKernelGGL((k_pairs<R, PSI, 4>), grid, block, 0, p->stream, N, p->nc, per, L, rc, alpha,
                           nperm, x, off, fil, cs, sp, q, base, out);
    else
        hipLaunchKernelGGL((k_pairs<R, PSI, 1>), grid, block, 0, p->stream, N, p->nc, per, L, rc, alpha,
                           nperm, x, off, fil, cs, sp, q, base, out);
}

void launch_pairs(bs_plan_t p, int psi, const double *base, double *out, bool alone) {
    if (p->fp32) {
        if (psi) pairs_r<float, true>(p, base, out, alone);
        else pairs_r<float, false>(p, base, out, alone);
    } else {
        if (psi) pairs_r<double, true>(p, base, out, alone);
        else pairs_r<double, false>(p, base, out, alone);
    }
}

// ------------------------------------------------------------------ energy
// E = (1/2V) sum_l Gamma_l oint psi . ds (eq:kinetic_energy_streamfunction)
// with psi between the nodes given by the spline through its nodal values on
// the curve's own knots (slopes eD, quintic second derivatives eS) and the
// curve's Q-point rule on every segment: sum over quadrature points of
// psi(tau_q) . q_q, the vector charges q_q = Gamma w dtau s'(tau_q).
// Partial sums per block; a second pass adds them in a fixed order.
constexpr int kRedBlock = 256;
constexpr int kEnergyMaxQ = 4;
struct GLNodes {
    double h[kEnergyMaxQ];
};

template <int ORDER>
__global__ void k_energy_partial(int N, int Q, const double *__restrict__ psi,
                                 const double *__restrict__ eD, const double *__restrict__ eS,
                                 const double *__restrict__ dtau, const int *__restrict__ off,
                                 const int *__restrict__ fil, const double *__restrict__ qchg,
                                 GLNodes gl, double *__restrict__ partial) {
    __shared__ double sh[kRedBlock];
    double s = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
        const int f = fil[j], jn = (j + 1 < off[f + 1]) ? j + 1 : off[f];
        SegPoly<ORDER> sp;
        sp.load(psi, psi, jn, eD, eS, j, jn, dtau[j]);
        for (int i = 0; i < Q; i++) {
            double pv[3];
            sp.pos(gl.h[i], pv);
            const double *c = qchg + 3 * ((size_t)j * Q + i);
            s += pv[0] * c[0] + pv[1] * c[1] + pv[2] * c[2];
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_energy_final(int nb, double scale, const double *__restrict__ partial,
                               double *__restrict__ e) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += partial[b];
        *e = s * scale;
    }
}

void launch_energy(bs_plan_t p, const double *psi, double *partial, int nblocks) {
    double L = p->prm.L;
    double *eD = (double *)p->e_D.p, *eS = (double *)p->e_S.p;
    launch_spline_data(p, psi, eD, eS);
    GLRule r = gl_rule(p->Q);
    GLNodes g;
    for (int i = 0; i < kEnergyMaxQ; i++) g.h[i] = r.h[i];
    auto kern = p->order == 6 ? k_energy_partial<6> : k_energy_partial<4>;
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kRedBlock), 0, p->stream, (int)p->N, p->Q, psi,
                       (const double *)eD, (const double *)eS, (const double *)p->d_dtau.p,
                       (const int *)p->d_off.p, (const int *)p->d_fil.p,
                       (const double *)p->d_qchg.p, g, partial);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, p->stream, nblocks,
                       1.0 / (2.0 * L * L * L), partial, partial + nblocks);
}

}  // namespace bs
