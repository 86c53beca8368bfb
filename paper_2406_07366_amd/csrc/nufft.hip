// Long-range part: type-1 NUFFT (spread + forward r2c FFT), the spectral
// operator, and type-2 NUFFT (inverse c2r FFT + interpolation), Sec. 3.3 and
// App. A.
//
// Spread (tile-owned, atomic-free in global memory): one workgroup owns a
// T^3 tile of the grid, accumulates every point whose w^3 stencil overlaps
// it into an LDS copy of the tile (LDS atomics), and writes the tile once.
// The grid is therefore written exactly once (no separate zeroing pass and
// no global atomics), which is what matters at the low point densities of
// filament tangles (~0.01-0.03 points per grid cell).
//
// Spectral operator, per retained mode k = 2 pi m / L with |m_i| <= K, k != 0:
//   v_hat = i k x G_hat exp(-k^2/(4 alpha^2)) / (k^2 L^3 F(m_x)^2 F(m_y)^2 F(m_z)^2)
// (eq:velocity_longrange_physical; psi_hat without the i k x), where G_hat is
// the unnormalised DFT of the spread grid and F(m) = (w/2) phi_hat(pi m w / n)
// is the kernel's transform per axis (one factor undoes the spreading, the
// other pre-compensates the interpolation).  Every other mode is set to 0
// (k = 0 by zero net vorticity; |m_i| > K by truncation).
#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

// ----------------------------------------------------------------- spread
// Candidates (points whose stencil base lies in one of the nbv^3 bins that
// can reach this tile) are staged in LDS in batches of kSpreadBatch by all
// threads at once.  Each wavefront then takes candidates in turn; its lanes
// cover the (kx, ky) columns of the stencil (so the 64 lanes of one LDS
// instruction touch distinct, mostly consecutive words) and loop over kz.
// Every wavefront accumulates into its own LDS copy of the tile with plain
// adds (lanes never collide within an instruction), and the copies are summed
// in wavefront order when the tile is written: no atomics, and the summation
// order is fixed, so the grid is bitwise reproducible.
constexpr int kSpreadBatch = 64;
constexpr int kSpreadWaves = 4;

// Stencil cells k in [0, W) whose local index (d + k) mod n, d = base - t0,
// falls inside [0, TT): a contiguous range [lo, hi) (empty if hi <= lo).
template <int W, int TT>
__device__ __forceinline__ void overlap_range_t(int d, int n, int &lo, int &hi) {
    if (d < 0) d += n;                 // d in [0, n)
    if (d < TT) { lo = 0; hi = TT - d < W ? TT - d : W; }
    else {                              // stencil starts before the tile (wrap)
        lo = n - d;
        hi = lo + TT < W ? lo + TT : W;
    }
}
#define overlap_range(d, n, lo, hi) overlap_range_t<W, TT>(d, n, lo, hi)

template <typename R, int W, int TT>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread(int n, int NT, int nbv,
                                                              const int *__restrict__ start,
                                                              const int4 *__restrict__ base,
                                                              const R *__restrict__ ker,
                                                              const R *__restrict__ q,
                                                              R *__restrict__ grid) {
    constexpr int T3 = TT * TT * TT;
    constexpr int CB = kSpreadBatch;
    // stencil-base bins a tile can be reached from: nb per axis
    constexpr int NBMAX = 1 + (W - 1 + TT - 1) / TT;
    constexpr int NB3 = NBMAX * NBMAX * NBMAX;
    static_assert(NB3 <= 64 * kSpreadWaves, "bin table must fit one thread per bin");
    __shared__ R acc[kSpreadWaves][3 * T3];
    __shared__ R sker[CB * 3 * W];
    __shared__ R sq[CB * 3];
    __shared__ int4 sb[CB];
    __shared__ int bin_s[NB3], bin_o[NB3 + 1];
    const int tile = blockIdx.x;
    const int tx = tile % NT, ty = (tile / NT) % NT, tz = tile / (NT * NT);
    const int t0x = tx * TT, t0y = ty * TT, t0z = tz * TT;
    for (int i = threadIdx.x; i < kSpreadWaves * 3 * T3; i += blockDim.x) (&acc[0][0])[i] = (R)0;
    const int nbins = nbv * nbv * nbv;   // nbv <= NBMAX (checked by the launcher)
    if (threadIdx.x < nbins) {
        int i = threadIdx.x;
        int dx = i % nbv, dy = (i / nbv) % nbv, dz = i / (nbv * nbv);
        int bz = tz - dz; if (bz < 0) bz += NT;
        int by = ty - dy; if (by < 0) by += NT;
        int bx = tx - dx; if (bx < 0) bx += NT;
        int bin = (bz * NT + by) * NT + bx;
        bin_s[i] = start[bin];
        bin_o[i + 1] = start[bin + 1] - start[bin];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bin_o[0] = 0;
        for (int i = 0; i < nbins; i++) bin_o[i + 1] += bin_o[i];
    }
    __syncthreads();
    const int total = bin_o[nbins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    R *my = acc[wave];
    for (int c0 = 0; c0 < total; c0 += CB) {
        const int cn = total - c0 < CB ? total - c0 : CB;
        for (int i = threadIdx.x; i < cn * (3 * W + 4); i += blockDim.x) {
            int c = i / (3 * W + 4), k = i % (3 * W + 4);
            int ci = c0 + c, b = 0;
            while (bin_o[b + 1] <= ci) b++;
            int g = bin_s[b] + (ci - bin_o[b]);
            if (k < 3 * W) sker[c * 3 * W + k] = ker[(size_t)g * 3 * W + k];
            else if (k < 3 * W + 3) sq[c * 3 + (k - 3 * W)] = q[4 * (size_t)g + (k - 3 * W)];
            else sb[c] = base[g];
        }
        __syncthreads();
        for (int c = wave; c < cn; c += kSpreadWaves) {
            const int4 b = sb[c];
            int klo[3], khi[3];
            overlap_range(b.x - t0x, n, klo[0], khi[0]);
            overlap_range(b.y - t0y, n, klo[1], khi[1]);
            overlap_range(b.z - t0z, n, klo[2], khi[2]);
            if (khi[0] <= klo[0] || khi[1] <= klo[1] || khi[2] <= klo[2]) continue;
            const int ox = khi[0] - klo[0], oy = khi[1] - klo[1];
            const R *kp = sker + c * 3 * W;
            const R qx = sq[3 * c], qy = sq[3 * c + 1], qz = sq[3 * c + 2];
            // local index of stencil cell k along an axis: (b + k - t0) mod n
            int lx0 = b.x - t0x; if (lx0 < 0) lx0 += n;
            int ly0 = b.y - t0y; if (ly0 < 0) ly0 += n;
            int lz0 = b.z - t0z; if (lz0 < 0) lz0 += n;
            for (int l = lane; l < ox * oy; l += 64) {
                const int kx = klo[0] + l % ox, ky = klo[1] + l / ox;
                int lx = lx0 + kx; if (lx >= n) lx -= n;
                int ly = ly0 + ky; if (ly >= n) ly -= n;
                const R cxy = kp[kx] * kp[W + ky];
                const R cx = qx * cxy, cy = qy * cxy, cz = qz * cxy;
                R *col = my + ly * TT + lx;
                for (int kz = klo[2]; kz < khi[2]; kz++) {
                    int lz = lz0 + kz; if (lz >= n) lz -= n;
                    const R ph = kp[2 * W + kz];
                    R *cell = col + lz * TT * TT;
                    cell[0] += cx * ph;
                    cell[T3] += cy * ph;
                    cell[2 * T3] += cz * ph;
                }
            }
        }
        __syncthreads();
    }
    const size_t n3 = (size_t)n * n * n;
    for (int i = threadIdx.x; i < T3; i += blockDim.x) {
        int lx = i % TT, ly = (i / TT) % TT, lz = i / (TT * TT);
        size_t g = ((size_t)(t0z + lz) * n + (t0y + ly)) * n + (t0x + lx);
        R s0 = acc[0][i], s1 = acc[0][T3 + i], s2 = acc[0][2 * T3 + i];
#pragma unroll
        for (int w2 = 1; w2 < kSpreadWaves; w2++) {
            s0 += acc[w2][i]; s1 += acc[w2][T3 + i]; s2 += acc[w2][2 * T3 + i];
        }
        grid[g] = s0;
        grid[n3 + g] = s1;
        grid[2 * n3 + g] = s2;
    }
}

template <typename R, int TT>
static void spread_tt(bs_plan_t p) {
    const int w = p->prm.w;
    int nb = 1 + ceil_div(w - 1, TT);   // equals the kernel's NBMAX for W = w
    int nbv = nb < p->NT ? nb : p->NT;
    if (nbv * nbv * nbv > 256) return;  // unreachable for w <= 16, TT >= 4
    dim3 grid(p->NT * p->NT * p->NT), block(64 * kSpreadWaves);
    const int *start = (const int *)p->sp_start.p;
    const int4 *base = (const int4 *)p->sp_base.p;
    const R *ker = (const R *)p->sp_ker.p, *q = (const R *)p->sp_q.p;
    R *g = (R *)p->grid.p;
#define SPREAD_CASE(WW) \
    case WW: hipLaunchKernelGGL((k_spread<R, WW, TT>), grid, block, 0, p->stream, p->n, p->NT, nbv, start, base, ker, q, g); break;
    switch (w) {
        SPREAD_CASE(4) SPREAD_CASE(5) SPREAD_CASE(6) SPREAD_CASE(7) SPREAD_CASE(8)
        SPREAD_CASE(9) SPREAD_CASE(10) SPREAD_CASE(11) SPREAD_CASE(12) SPREAD_CASE(13)
        SPREAD_CASE(14) SPREAD_CASE(15) SPREAD_CASE(16)
        default: break;
    }
#undef SPREAD_CASE
}

void launch_spread(bs_plan_t p) {
    if (p->fp32) {
        if (p->T == 8) spread_tt<float, 8>(p); else spread_tt<float, 4>(p);
    } else {
        if (p->T == 8) spread_tt<double, 8>(p); else spread_tt<double, 4>(p);
    }
}

// ------------------------------------------------------------------- FFTs
int fft_forward(bs_plan_t p) {
    hipfftResult r;
    if (p->fp32) r = hipfftExecR2C(p->fft_fwd, (hipfftReal *)p->grid.p, (hipfftComplex *)p->spec.p);
    else r = hipfftExecD2Z(p->fft_fwd, (hipfftDoubleReal *)p->grid.p, (hipfftDoubleComplex *)p->spec.p);
    if (r != HIPFFT_SUCCESS) return set_error(p, BS_EDEVICE, "hipfft forward transform failed");
    return BS_OK;
}

int fft_inverse(bs_plan_t p) {
    hipfftResult r;
    if (p->fp32) r = hipfftExecC2R(p->fft_inv, (hipfftComplex *)p->spec.p, (hipfftReal *)p->grid.p);
    else r = hipfftExecZ2D(p->fft_inv, (hipfftDoubleComplex *)p->spec.p, (hipfftDoubleReal *)p->grid.p);
    if (r != HIPFFT_SUCCESS) return set_error(p, BS_EDEVICE, "hipfft inverse transform failed");
    return BS_OK;
}

// ------------------------------------------------------- spectral operator
template <typename R>
__global__ void k_spectral(int n, int K, int psi, double k0, double inv4a2, double invV,
                           const double *__restrict__ dec2, R *__restrict__ spec) {
    const int nh = n / 2 + 1;
    const size_t nc = (size_t)n * n * nh;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    int ix = (int)(idx % nh), iy = (int)((idx / nh) % n), iz = (int)(idx / ((size_t)nh * n));
    int mx = ix, my = iy <= n / 2 ? iy : iy - n, mz = iz <= n / 2 ? iz : iz - n;
    int ax = mx, ay = my < 0 ? -my : my, az = mz < 0 ? -mz : mz;
    R *G0 = spec + 2 * idx, *G1 = spec + 2 * (nc + idx), *G2 = spec + 2 * (2 * nc + idx);
    if (ax > K || ay > K || az > K || (ax == 0 && ay == 0 && az == 0)) {
        G0[0] = G0[1] = G1[0] = G1[1] = G2[0] = G2[1] = (R)0;
        return;
    }
    double kx = k0 * mx, ky = k0 * my, kz = k0 * mz;
    double k2 = kx * kx + ky * ky + kz * kz;
    double f = exp(-k2 * inv4a2) / k2 * invV * dec2[ax] * dec2[ay] * dec2[az];
    R gr[3] = {G0[0], G1[0], G2[0]}, gi[3] = {G0[1], G1[1], G2[1]};
    if (psi) {
        R fr = (R)f;
        G0[0] = gr[0] * fr; G0[1] = gi[0] * fr;
        G1[0] = gr[1] * fr; G1[1] = gi[1] * fr;
        G2[0] = gr[2] * fr; G2[1] = gi[2] * fr;
        return;
    }
    // c = k x G (complex), result = i c f = (-Im c, Re c) f
    R fkx = (R)(kx * f), fky = (R)(ky * f), fkz = (R)(kz * f);
    R cr0 = fky * gr[2] - fkz * gr[1], ci0 = fky * gi[2] - fkz * gi[1];
    R cr1 = fkz * gr[0] - fkx * gr[2], ci1 = fkz * gi[0] - fkx * gi[2];
    R cr2 = fkx * gr[1] - fky * gr[0], ci2 = fkx * gi[1] - fky * gi[0];
    G0[0] = -ci0; G0[1] = cr0;
    G1[0] = -ci1; G1[1] = cr1;
    G2[0] = -ci2; G2[1] = cr2;
}

void launch_spectral(bs_plan_t p, int psi) {
    const int n = p->n;
    size_t nc = (size_t)n * n * (n / 2 + 1);
    double L = p->prm.L;
    double k0 = 2.0 * kPi / L, inv4a2 = 1.0 / (4.0 * p->prm.alpha * p->prm.alpha);
    double invV = 1.0 / (L * L * L);
    const double *dec2 = (const double *)p->deconv.p + (p->prm.K + 1);
    unsigned nb = (unsigned)((nc + 255) / 256);
    if (p->fp32)
        hipLaunchKernelGGL(k_spectral<float>, dim3(nb), dim3(256), 0, p->stream, n, p->prm.K, psi,
                           k0, inv4a2, invV, dec2, (float *)p->spec.p);
    else
        hipLaunchKernelGGL(k_spectral<double>, dim3(nb), dim3(256), 0, p->stream, n, p->prm.K,
                           psi, k0, inv4a2, invV, dec2, (double *)p->spec.p);
}

// ------------------------------------------------------ vorticity modes
// omega_hat(m) = G_hat(m) / (L^3 F(m_x) F(m_y) F(m_z)) for the half space of
// modes, from the r2c layout (m_x >= 0 stored; m_x < 0 by conjugation).
template <typename R>
__global__ void k_modes(int n, int K, double invV, const double *__restrict__ dec1,
                        const R *__restrict__ spec, double *__restrict__ out) {
    const int W = 2 * K + 1;
    const int nh = n / 2 + 1;
    const size_t nc = (size_t)n * n * nh;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (K + 1) * W * W) return;
    int mx = t % W - K, my = (t / W) % W - K, mz = t / (W * W);
    bool in_half = (mz > 0) || (mz == 0 && (my > 0 || (my == 0 && mx > 0)));
    double *o = out + 6 * (size_t)t;
    if (!in_half) {
        for (int c = 0; c < 6; c++) o[c] = 0.0;
        return;
    }
    int sx = mx, sy = my, sz = mz;
    double sgn = 1.0;
    if (mx < 0) { sx = -mx; sy = -my; sz = -mz; sgn = -1.0; }
    int iy = sy < 0 ? sy + n : sy, iz = sz < 0 ? sz + n : sz;
    size_t idx = ((size_t)iz * n + iy) * nh + sx;
    double f = invV * dec1[mx < 0 ? -mx : mx] * dec1[my < 0 ? -my : my] * dec1[mz];
    for (int c = 0; c < 3; c++) {
        o[2 * c] = (double)spec[2 * (c * nc + idx)] * f;
        o[2 * c + 1] = sgn * (double)spec[2 * (c * nc + idx) + 1] * f;
    }
}

void launch_modes(bs_plan_t p, double *out) {
    int K = p->prm.K, W = 2 * K + 1;
    double L = p->prm.L;
    const double *dec1 = (const double *)p->deconv.p;
    int tot = (K + 1) * W * W;
    if (p->fp32)
        hipLaunchKernelGGL(k_modes<float>, dim3(ceil_div(tot, 256)), dim3(256), 0, p->stream, p->n,
                           K, 1.0 / (L * L * L), dec1, (const float *)p->spec.p, out);
    else
        hipLaunchKernelGGL(k_modes<double>, dim3(ceil_div(tot, 256)), dim3(256), 0, p->stream,
                           p->n, K, 1.0 / (L * L * L), dec1, (const double *)p->spec.p, out);
}

// ---------------------------------------------------------- interpolation
// G lanes per node; lane l sums the x-rows (ky, kz) = (r % W, r / W) for
// r = l, l + G, ...; partial sums combined by a fixed xor-shuffle tree.
template <typename R, int W, int G>
__global__ __launch_bounds__(256) void k_interp(int N, const int *__restrict__ perm,
                                                const double *__restrict__ x, double L,
                                                double inv_h, int n, double zeta, double inv_den,
                                                const R *__restrict__ grid,
                                                double *__restrict__ out) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gid / G, lane = gid % G;
    if (t >= N) return;
    const int o = perm[t];
    const double half = 0.5 * W;
    double fx, fy, fz;
    int bx = stencil_base(wrap_box(x[3 * o], L), inv_h, W, n, &fx);
    int by = stencil_base(wrap_box(x[3 * o + 1], L), inv_h, W, n, &fy);
    int bz = stencil_base(wrap_box(x[3 * o + 2], L), inv_h, W, n, &fz);
    int ix[W];
    R px[W];
#pragma unroll
    for (int k = 0; k < W; k++) {
        int c = bx + k;
        ix[k] = c >= n ? c - n : c;
        px[k] = (R)kb_phi((k - fx) / half, zeta, inv_den);
    }
    const size_t n3 = (size_t)n * n * n;
    R a0 = 0, a1 = 0, a2 = 0;
    for (int r = lane; r < W * W; r += G) {
        int ky = r % W, kz = r / W;
        int cy = by + ky; cy = cy >= n ? cy - n : cy;
        int cz = bz + kz; cz = cz >= n ? cz - n : cz;
        R wyz = (R)(kb_phi((ky - fy) / half, zeta, inv_den) * kb_phi((kz - fz) / half, zeta, inv_den));
        const R *row = grid + ((size_t)cz * n + cy) * n;
        R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int kx = 0; kx < W; kx++) {
            int c = ix[kx];
            s0 += px[kx] * row[c];
            s1 += px[kx] * row[n3 + c];
            s2 += px[kx] * row[2 * n3 + c];
        }
        a0 += wyz * s0; a1 += wyz * s1; a2 += wyz * s2;
    }
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) {
        a0 += __shfl_xor(a0, m, G);
        a1 += __shfl_xor(a1, m, G);
        a2 += __shfl_xor(a2, m, G);
    }
    if (lane == 0) {
        out[3 * o] += (double)a0;
        out[3 * o + 1] += (double)a1;
        out[3 * o + 2] += (double)a2;
    }
}

constexpr int kInterpLanes = 64;

template <typename R>
static void interp_r(bs_plan_t p, double *out) {
    const int N = (int)p->N;
    dim3 grid(ceil_div((int64_t)N * kInterpLanes, 256)), block(256);
    const double L = p->prm.L, inv_h = p->n / L, zeta = p->prm.zeta;
    const double inv_den = 1.0 / (-expm1(-2.0 * zeta));
    const int *perm = (const int *)p->nd_perm.p;
    const double *x = (const double *)p->d_x.p;
    const R *g = (const R *)p->grid.p;
#define INTERP_CASE(WW) \
    case WW: hipLaunchKernelGGL((k_interp<R, WW, kInterpLanes>), grid, block, 0, p->stream, N, perm, x, L, inv_h, p->n, zeta, inv_den, g, out); break;
    switch (p->prm.w) {
        INTERP_CASE(4) INTERP_CASE(5) INTERP_CASE(6) INTERP_CASE(7) INTERP_CASE(8)
        INTERP_CASE(9) INTERP_CASE(10) INTERP_CASE(11) INTERP_CASE(12) INTERP_CASE(13)
        INTERP_CASE(14) INTERP_CASE(15) INTERP_CASE(16)
        default: break;
    }
#undef INTERP_CASE
}

void launch_interp(bs_plan_t p, double *out) {
    if (p->fp32) interp_r<float>(p, out);
    else interp_r<double>(p, out);
}

}  // namespace bs
