// Long-range part: type-1 NUFFT (spread + forward r2c FFT), the spectral
// operator, and type-2 NUFFT (inverse c2r FFT + interpolation), Sec. 3.3 and
// App. A.
//
// Spread (tile-owned, atomic-free): one wavefront owns a T^3 tile of the
// grid, accumulates every point whose w^3 stencil overlaps it in registers,
// and writes the tile once.  The grid is therefore written exactly once (no
// zeroing pass, no atomics), which is what matters at the low point
// densities of filament tangles (~0.01-0.03 points per grid cell).
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
// One wavefront owns a T^3 tile of the grid and accumulates it in registers.
// Candidates are the points whose stencil base lies in one of the nbv^3
// bins that can reach the tile.  They are staged 64 at a time (lane c loads
// candidate c), and the candidates that overlap the tile are compacted into
// LDS with a ballot, in candidate order.  Each grid cell is written exactly
// once, with no atomics and a fixed summation order (bitwise reproducible),
// and the LDS holds only the staged candidates.
//
// T = 8, one wavefront per tile (matrix cores): the tile's sum over its
// candidates p is a matrix product, G[(c, z)][(y, x)] =
// sum_p A[(c, z)][p] B[p][(y, x)] with A = q_c wz[z] (24 rows) and
// B = wy[y] wx[x] (64 columns), so it runs on v_mfma_*_16x16x4, four
// candidates per instruction: rows padded to 32 (row block 0: c = 0, 1;
// block 1: c = 2 and 8 zero rows), columns in 4 blocks of two y rows.  Per 4
// candidates a lane reads 9 staged values and issues 8 MFMAs (the vector form
// reads 13 values per candidate for its 24 FMAs).  The kernel values are
// staged as they are, with each axis's offset into the tile, so that a
// lane's loads of base, kernel values and charge go out together: the time
// of a tile is mostly the latency of its two rounds of global loads (bin
// starts, then candidates).
//
// Vector form (T = 4, and tiles split over several wavefronts on small
// grids): lane c turns its candidate's kernel values into the tile's frame
// (T weights per axis, zero where the stencil misses the tile) before
// staging; lane l owns the columns (lx, ly) = (l % T, (l / T) % T) over
// ZL = T^3 / 64 z cells from (l / T^2) ZL and adds q wx[lx] wy[ly] wz[z] per
// candidate; the partial tiles of the wavefronts are summed in LDS.
//
// Tiles are spread over the 8 XCDs in contiguous ranges (blocks b, b+8, ...
// run on one XCD), so neighbouring tiles, which share candidate bins and the
// cache lines of their grid rows, go through the same L2.
//
template <typename R> struct Mfma4;
template <> struct Mfma4<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V op(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ constexpr int row(int k4, int v) { return k4 + 4 * v; }
};
template <> struct Mfma4<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ V op(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ constexpr int row(int k4, int v) { return 4 * k4 + v; }
};

template <typename R, int W, int TT, int WAVES, bool MMA>
__global__ __launch_bounds__(64 * WAVES) void k_spread(int n, int NT, int nbv, int per_xcd,
                                                       const int *__restrict__ start,
                                                       const int4 *__restrict__ base,
                                                       const R *__restrict__ ker,
                                                       const R *__restrict__ q,
                                                       R *__restrict__ grid) {
    constexpr int T3 = TT * TT * TT;
    constexpr int ZL = T3 / 64;
    // staged words per candidate: the vector form stages T weights per axis
    // in the tile's frame, the MMA form the W kernel values per axis as they
    // are (with the stencil index of the tile's first cell per axis in soff);
    // both then q and a pad
    constexpr int SW = MMA ? 3 * W + 4 : 3 * TT + 4;
    constexpr int NBMAX = 1 + (W - 1 + TT - 1) / TT;   // bins per axis that reach a tile
    constexpr int NB3 = NBMAX * NBMAX * NBMAX;
    // staging area per wavefront; reused for the sum over wavefronts
    constexpr int STAGE = WAVES * 64 * SW, RED = WAVES > 1 ? WAVES * 3 * T3 : 0;
    __shared__ R lds[STAGE > RED ? STAGE : RED];
    __shared__ int bin_s[NB3], bin_o[NB3], bin_total;
    __shared__ int soff[MMA ? WAVES * 64 : 1];
    const int ntiles = NT * NT * NT;
    const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int tx = tile % NT, ty = (tile / NT) % NT, tz = tile / (NT * NT);
    const int t0[3] = {tx * TT, ty * TT, tz * TT};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lx = lane % TT, ly = (lane / TT) % TT, lz0 = (lane / (TT * TT)) * ZL;
    static_assert(!MMA || (TT == 8 && WAVES == 1), "the matrix-core form: 8^3 tiles, one wavefront");
    typedef typename Mfma4<R>::V V4;
    const int i16 = lane & 15, k4 = lane >> 4;
    R acc[3][ZL];
    V4 dacc[2][4];   // [row block][column block] (MMA form)
#pragma unroll
    for (int z = 0; z < ZL; z++) acc[0][z] = acc[1][z] = acc[2][z] = (R)0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) dacc[a][b] = V4{(R)0, (R)0, (R)0, (R)0};
    // start of each bin and exclusive prefix of the bin sizes, in LDS
    // (bins taken 64 at a time by wavefront 0, prefix by shuffles)
    const int nbins = nbv * nbv * nbv;   // nbv <= NBMAX (checked by the launcher)
    if (wave == 0) {
        int total = 0;
        for (int i0 = 0; i0 < nbins; i0 += 64) {
            const int i = i0 + lane;
            int bstart = 0, bsize = 0;
            if (i < nbins) {
                const int dx = i % nbv, dy = (i / nbv) % nbv, dz = i / (nbv * nbv);
                int bz = tz - dz; if (bz < 0) bz += NT;
                int by = ty - dy; if (by < 0) by += NT;
                int bx = tx - dx; if (bx < 0) bx += NT;
                const int bin = (bz * NT + by) * NT + bx;
                bstart = start[bin];
                bsize = start[bin + 1] - bstart;
            }
            int incl = bsize;
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(incl, d);
                if (lane >= d) incl += v;
            }
            if (i < nbins) { bin_s[i] = bstart; bin_o[i] = total + incl - bsize; }
            total += __shfl(incl, 63);
        }
        if (lane == 0) bin_total = total;
    }
    __syncthreads();
    const int total = bin_total;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // wavefront w takes chunks w, w + WAVES, ...; every wavefront runs the
    // same number of rounds so that the block barriers match
    const int nchunks = (total + 63) / 64;
    const int rounds = (nchunks + WAVES - 1) / WAVES;
    R *st = lds + wave * 64 * SW;
    for (int rd = 0; rd < rounds; rd++) {
        const int ci = (rd * WAVES + wave) * 64 + lane;
        // bin of candidate ci: the last bin whose exclusive prefix is <= ci
        int b = 0;
        for (int step = 64; step > 0; step >>= 1) {
            const int tb = b + step;
            if (tb < nbins && bin_o[tb] <= ci) b = tb;
        }
        const int g = bin_s[b] + (ci - bin_o[b]);
        unsigned long long m;
        if constexpr (MMA) {
            // the candidate's base, kernel values and charge, all loaded at
            // once; offset o of axis a = stencil index of the tile's first
            // cell, in [1 - T, W - 1] when the stencil reaches the tile (one
            // interval: the plan keeps n >= W + T)
            R kv[3 * W], qv[3];
            int offp = 0;
            bool act = false;
            if (ci < total) {
                const int4 bb = base[g];
                const R *kg = ker + (size_t)g * 3 * W;
#pragma unroll
                for (int j = 0; j < 3 * W; j++) kv[j] = kg[j];
#pragma unroll
                for (int c = 0; c < 3; c++) qv[c] = q[4 * (size_t)g + c];
                const int bv[3] = {bb.x, bb.y, bb.z};
                act = true;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    int off = t0[a] - bv[a];
                    if (off < 0) off += n;
                    const int o = off < W ? off : off - n;
                    act = act && o > -TT;
                    offp |= (o + TT) << (5 * a);
                }
            }
            m = __ballot(act);
            if (act) {
                const int slot = __popcll(m & below);
                R *s = st + slot * SW;
#pragma unroll
                for (int j = 0; j < 3 * W; j++) s[j] = kv[j];
#pragma unroll
                for (int c = 0; c < 3; c++) s[3 * W + c] = qv[c];
                soff[wave * 64 + slot] = offp;
            }
        } else {
            R wgt[3][TT];
            bool act = false;
            if (ci < total) {
                const int4 bb = base[g];
                const int bv[3] = {bb.x, bb.y, bb.z};
                act = true;
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    // stencil index of the tile's first cell along axis a
                    int off = t0[a] - bv[a];
                    if (off < 0) off += n;
                    bool any = false;
#pragma unroll
                    for (int l = 0; l < TT; l++) {
                        int k = off + l;
                        if (k >= n) k -= n;
                        R wv = (R)0;
                        if (k < W) { wv = ker[((size_t)g * 3 + a) * W + k]; any = true; }
                        wgt[a][l] = wv;
                    }
                    act = act && any;
                }
            }
            m = __ballot(act);
            if (act) {
                R *s = st + __popcll(m & below) * SW;
#pragma unroll
                for (int a = 0; a < 3; a++)
#pragma unroll
                    for (int l = 0; l < TT; l++) s[a * TT + l] = wgt[a][l];
                s[3 * TT] = q[4 * (size_t)g];
                s[3 * TT + 1] = q[4 * (size_t)g + 1];
                s[3 * TT + 2] = q[4 * (size_t)g + 2];
            }
        }
        __syncthreads();
        const int na = __popcll(m);
        if constexpr (MMA) {
            // candidates 4 at a time: A[(c, z)][k] = q_c wz[z] (rows 0..15: c = 0, 1;
            // rows 16..23: c = 2; rows 24..31 zero), B[k][(y, x)] = wy[y] wx[x]
            // (column block b: y = 2b, 2b + 1), the weight of tile cell l
            // along an axis being kernel value o + l (zero outside 0..W-1);
            // a missing candidate gives zero rows
            for (int c0 = 0; c0 < na; c0 += 4) {
                const int c = c0 + k4;
                R a0 = (R)0, a1 = (R)0, bv[4] = {(R)0, (R)0, (R)0, (R)0};
                if (c < na) {
                    const R *s = st + c * SW;
                    const int op = soff[wave * 64 + c];
                    const int kx = (op & 31) - TT + (i16 & 7), ky = ((op >> 5) & 31) - TT + (i16 >> 3),
                              kz = ((op >> 10) & 31) - TT + (i16 & 7);
                    const R wx = (unsigned)kx < (unsigned)W ? s[kx] : (R)0;
                    const R wz = (unsigned)kz < (unsigned)W ? s[2 * W + kz] : (R)0;
                    a0 = s[3 * W + (i16 >> 3)] * wz;
                    if (i16 < 8) a1 = s[3 * W + 2] * wz;
#pragma unroll
                    for (int b = 0; b < 4; b++) {
                        const int k = ky + 2 * b;
                        bv[b] = ((unsigned)k < (unsigned)W ? s[W + k] : (R)0) * wx;
                    }
                }
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    dacc[0][b] = Mfma4<R>::op(a0, bv[b], dacc[0][b]);
                    dacc[1][b] = Mfma4<R>::op(a1, bv[b], dacc[1][b]);
                }
            }
        } else {
            for (int c = 0; c < na; c++) {
                const R *s = st + c * SW;
                const R wxy = s[lx] * s[TT + ly];
                const R qx = s[3 * TT] * wxy, qy = s[3 * TT + 1] * wxy, qz = s[3 * TT + 2] * wxy;
#pragma unroll
                for (int z = 0; z < ZL; z++) {
                    const R wz = s[2 * TT + lz0 + z];
                    acc[0][z] += qx * wz;
                    acc[1][z] += qy * wz;
                    acc[2][z] += qz * wz;
                }
            }
        }
        __syncthreads();
    }
    const size_t n3 = (size_t)n * n * n;
    if constexpr (MMA) {
        // result element (row block a, column block b, v): row r = 16 a + row(k4, v)
        // (component r / 8, z = r % 8; rows 24..31 are padding), column
        // 16 b + i16 (y = 2 b + i16 / 8, x = i16 % 8)
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int r = 16 * a + Mfma4<R>::row(k4, v);
                    if (r < 24) {
                        const size_t gi = ((size_t)(t0[2] + (r & 7)) * n + (t0[1] + 2 * b + (i16 >> 3))) * n +
                                          (t0[0] + (i16 & 7));
                        grid[(size_t)(r >> 3) * n3 + gi] = dacc[a][b][v];
                    }
                }
        return;
    }
    if (WAVES > 1) {
        // cell (lx, ly, lz0 + z) of wavefront w's partial tile
#pragma unroll
        for (int z = 0; z < ZL; z++) {
            const int cell = ((lz0 + z) * TT + ly) * TT + lx;
            for (int c = 0; c < 3; c++) lds[(wave * 3 + c) * T3 + cell] = acc[c][z];
        }
        __syncthreads();
        if (wave != 0) return;
#pragma unroll
        for (int z = 0; z < ZL; z++) {
            const int cell = ((lz0 + z) * TT + ly) * TT + lx;
            for (int c = 0; c < 3; c++) {
                R v = lds[c * T3 + cell];
                for (int w2 = 1; w2 < WAVES; w2++) v += lds[(w2 * 3 + c) * T3 + cell];
                acc[c][z] = v;
            }
        }
    }
#pragma unroll
    for (int z = 0; z < ZL; z++) {
        const size_t gi = ((size_t)(t0[2] + lz0 + z) * n + (t0[1] + ly)) * n + (t0[0] + lx);
        grid[gi] = acc[0][z];
        grid[n3 + gi] = acc[1][z];
        grid[2 * n3 + gi] = acc[2][z];
    }
}

// grids with fewer tiles than this split each tile's candidates over 4
// wavefronts (more parallelism for small grids), and float32 grids of at most
// kSpreadWideTiles tiles over 8 (a 64^3 grid of 8^3 tiles: the busiest tile
// holds ~5x the mean candidate count).  The float64 variant stays at 4: at 8
// its staging area (112 KB) leaves one workgroup per CU
constexpr int kSpreadSplitTiles = 8192;
constexpr int kSpreadWideTiles = 512;

template <typename R, int TT>
static void spread_tt(bs_plan_t p) {
    const int w = p->prm.w;
    int nb = 1 + ceil_div(w - 1, TT);
    int nbv = nb < p->NT ? nb : p->NT;
    if (nbv > nb) return;   // the kernel's bin table holds nb^3 bins
    const int ntiles = p->NT * p->NT * p->NT;
    const int per = ceil_div(ntiles, 8);
    const bool split = ntiles < kSpreadSplitTiles;
    const bool wide = sizeof(R) == 4 && TT == 8 && ntiles <= kSpreadWideTiles;
    dim3 grid(8 * per), block(wide ? 512 : (split ? 256 : 64));
    const int *start = (const int *)p->sp_start.p;
    const int4 *base = (const int4 *)p->sp_base.p;
    const R *ker = (const R *)p->sp_ker.p, *q = (const R *)p->sp_q.p;
    R *g = (R *)p->grid.p;
#define SPREAD_CASE(WW)                                                                          \
    case WW:                                                                                     \
        if constexpr (sizeof(R) == 4) {                                                          \
            if (wide) {                                                                          \
                hipLaunchKernelGGL((k_spread<R, WW, TT, 8, false>), grid, block, 0, p->stream,   \
                                   p->n, p->NT, nbv, per, start, base, ker, q, g);               \
                break;                                                                           \
            }                                                                                    \
        }                                                                                        \
        if (split)                                                                               \
            hipLaunchKernelGGL((k_spread<R, WW, TT, 4, false>), grid, block, 0, p->stream, p->n, \
                               p->NT, nbv, per, start, base, ker, q, g);                         \
        else                                                                                     \
            hipLaunchKernelGGL((k_spread<R, WW, TT, 1, TT == 8>), grid, block, 0, p->stream,     \
                               p->n, p->NT, nbv, per, start, base, ker, q, g);                   \
        break;
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
// G = 64 lanes per node.  Lane j < 3W evaluates the kernel value of stencil
// cell j % W along axis j / W once; the others read them by shuffles.  Lane
// l owns the stencil columns (kx, ky) = (r % W, r / W) for r = l, l + G, ...
// and runs along z, so the lanes of one load instruction read W rows of W
// consecutive grid values (a few cache lines, not one line per lane).  The
// partial sums are combined by a fixed xor-shuffle tree.  Nodes come in
// pair-cell order, and consecutive blocks of them stay on one XCD (blocks
// b, b+8, ... run on one XCD), so the grid rows that neighbouring nodes share
// are fetched into one L2.
template <typename R, int W, int G, bool IL>
__global__ __launch_bounds__(256) void k_interp(int N, int per_xcd, const int *__restrict__ perm,
                                                const double *__restrict__ x, double L,
                                                double inv_h, int n, double zeta, double inv_den,
                                                const R *__restrict__ grid,
                                                const double *__restrict__ base,
                                                double *__restrict__ out) {
    static_assert(3 * W <= G, "one lane per kernel value");
    constexpr int NR = (W * W + G - 1) / G;
    const int blk = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    const int gid = blk * blockDim.x + threadIdx.x;
    const int t = gid / G, lane = gid % G;
    if (t >= N) return;   // whole wavefronts exit together
    const int o = perm[t];
    const double half = 0.5 * W;
    double f[3];
    int bb[3];
    for (int a = 0; a < 3; a++) bb[a] = stencil_base(wrap_box(x[3 * o + a], L), inv_h, W, n, &f[a]);
    R phi = (R)0;
    if (lane < 3 * W) {
        const int a = lane / W, k = lane % W;
        phi = (R)kb_phi((k - f[a]) / half, zeta, inv_den);
    }
    R pz[W];
    int iz[W];
#pragma unroll
    for (int k = 0; k < W; k++) {
        pz[k] = __shfl(phi, 2 * W + k, G);
        const int c = bb[2] + k;
        iz[k] = c >= n ? c - n : c;
    }
    R wxy[NR];
    size_t col[NR];
#pragma unroll
    for (int i = 0; i < NR; i++) {
        const int r = lane + i * G, rc = r < W * W ? r : 0;
        const int kx = rc % W, ky = rc / W;
        const R wx = __shfl(phi, kx, G), wy = __shfl(phi, W + ky, G);
        wxy[i] = r < W * W ? wx * wy : (R)0;
        int cx = bb[0] + kx; cx = cx >= n ? cx - n : cx;
        int cy = bb[1] + ky; cy = cy >= n ? cy - n : cy;
        col[i] = (size_t)cy * n + cx;
    }
    const size_t n2 = (size_t)n * n, n3 = n2 * n;
    R a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int i = 0; i < NR; i++) {
        if (lane + i * G < W * W) {
            // IL: components interleaved, [n][n][n][3]; else [3][n][n][n]
            const R *g = grid + (IL ? 3 : 1) * col[i];
            R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int kz = 0; kz < W; kz++) {
                if constexpr (IL) {
                    const size_t c = 3 * (size_t)iz[kz] * n2;
                    s0 += pz[kz] * g[c];
                    s1 += pz[kz] * g[c + 1];
                    s2 += pz[kz] * g[c + 2];
                } else {
                    const size_t c = (size_t)iz[kz] * n2;
                    s0 += pz[kz] * g[c];
                    s1 += pz[kz] * g[n3 + c];
                    s2 += pz[kz] * g[2 * n3 + c];
                }
            }
            a0 += wxy[i] * s0; a1 += wxy[i] * s1; a2 += wxy[i] * s2;
        }
    }
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) {
        a0 += __shfl_xor(a0, m, G);
        a1 += __shfl_xor(a1, m, G);
        a2 += __shfl_xor(a2, m, G);
    }
    if (lane == 0) {
        // base (if given) supplies the value the result is added to
        const double *b = base ? base : out;
        out[3 * o] = b[3 * o] + (double)a0;
        out[3 * o + 1] = b[3 * o + 1] + (double)a1;
        out[3 * o + 2] = b[3 * o + 2] + (double)a2;
    }
}

constexpr int kInterpLanes = 64;

template <typename R>
static void interp_r(bs_plan_t p, const double *base, double *out) {
    const int N = (int)p->N;
    const int nblk = ceil_div((int64_t)N * kInterpLanes, 256), per = ceil_div(nblk, 8);
    dim3 grid(8 * per), block(256);
    const double L = p->prm.L, inv_h = p->n / L, zeta = p->prm.zeta;
    const double inv_den = 1.0 / (-expm1(-2.0 * zeta));
    const int *perm = (const int *)p->nd_perm.p;
    const double *x = (const double *)p->d_x.p;
    const R *g = (const R *)p->grid.p;
    const bool il = grid_interleaved(p);
#define INTERP_CASE(WW) \
    case WW: \
        if (il) hipLaunchKernelGGL((k_interp<R, WW, kInterpLanes, true>), grid, block, 0, p->stream, N, per, perm, x, L, inv_h, p->n, zeta, inv_den, g, base, out); \
        else hipLaunchKernelGGL((k_interp<R, WW, kInterpLanes, false>), grid, block, 0, p->stream, N, per, perm, x, L, inv_h, p->n, zeta, inv_den, g, base, out); \
        break;
    switch (p->prm.w) {
        INTERP_CASE(4) INTERP_CASE(5) INTERP_CASE(6) INTERP_CASE(7) INTERP_CASE(8)
        INTERP_CASE(9) INTERP_CASE(10) INTERP_CASE(11) INTERP_CASE(12) INTERP_CASE(13)
        INTERP_CASE(14) INTERP_CASE(15) INTERP_CASE(16)
        default: break;
    }
#undef INTERP_CASE
}

void launch_interp(bs_plan_t p, const double *base, double *out) {
    if (p->fp32) interp_r<float>(p, base, out);
    else interp_r<double>(p, base, out);
}

}  // namespace bs
