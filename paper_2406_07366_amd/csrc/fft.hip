// Pruned 3-D transforms of the long-range step (Sec. 3.3) for power-of-two
// grids: only the retained modes |m_i| <= K (K < n/2) are ever formed or
// stored past the first transform of each direction, and the spectral
// operator is applied between the forward and inverse z transforms of the
// same columns, so it costs no pass of its own.
//
//   x forward   grid [3][n][n][n] real (x fastest)  ->  A [3][z][y][0..K]
//   y forward   A, FFT along y, keep my in [-K, K]  ->  B [3][my+K][z][0..K]
//   z fused     B, FFT along z, spectral operator (modes with |mz| > K, k = 0
//               zeroed), inverse FFT along z           ->  B (in place)
//   y inverse   B, zero-padded inverse FFT along y  ->  A [3][z][y][0..K]
//   x inverse   A, Hermitian c2r along x             ->  grid
//
// Conventions are those of an unnormalised r2c / c2r pair: forward
// exp(-2 pi i j m / n), inverse exp(+2 pi i j m / n), no scaling (the
// spectral operator carries 1/L^3 and the deconvolution).
//
// Each workgroup transforms a batch of sequences held in LDS with element j
// of sequence s at buf[j * nseq + s] (sequence index fastest, so the lanes of
// one butterfly step touch consecutive words).  Forward transforms are
// radix-2 decimation in time (bit-reversed input, natural output); inverse
// transforms are decimation in frequency (natural input, bit-reversed
// output), so no reordering pass is needed.
#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

template <typename R> struct Cx;
template <> struct Cx<float> { typedef float2 T; };
template <> struct Cx<double> { typedef double2 T; };

__device__ __forceinline__ int bitrev(int j, int logn) {
    return (int)(__brev((unsigned)j) >> (32 - logn));
}

// bit-reversed input -> natural output; tw[k] = exp(-2 pi i k / n), k < n/2
template <typename C>
__device__ void fft_dit(C *buf, int logn, int nseq, const C *__restrict__ tw) {
    const int hn = 1 << (logn - 1);
    for (int s = 1; s <= logn; s++) {
        const int lh = s - 1, half = 1 << lh, tsh = logn - s;
        for (int b = threadIdx.x; b < nseq * hn; b += blockDim.x) {
            const int seq = b % nseq, k = b / nseq;
            const int j = k & (half - 1), i0 = ((k >> lh) << (lh + 1)) + j, i1 = i0 + half;
            const C w = tw[j << tsh];
            C *p0 = buf + i0 * nseq + seq, *p1 = buf + i1 * nseq + seq;
            const C a = *p0, v = *p1;
            const C t = {w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x};
            *p0 = C{a.x + t.x, a.y + t.y};
            *p1 = C{a.x - t.x, a.y - t.y};
        }
        __syncthreads();
    }
}

// natural input -> bit-reversed output; tw[k] = exp(+2 pi i k / n), k < n/2
template <typename C>
__device__ void fft_dif(C *buf, int logn, int nseq, const C *__restrict__ tw) {
    const int hn = 1 << (logn - 1);
    for (int s = logn; s >= 1; s--) {
        const int lh = s - 1, half = 1 << lh, tsh = logn - s;
        for (int b = threadIdx.x; b < nseq * hn; b += blockDim.x) {
            const int seq = b % nseq, k = b / nseq;
            const int j = k & (half - 1), i0 = ((k >> lh) << (lh + 1)) + j, i1 = i0 + half;
            const C w = tw[j << tsh];
            C *p0 = buf + i0 * nseq + seq, *p1 = buf + i1 * nseq + seq;
            const C a = *p0, v = *p1;
            const C d = {a.x - v.x, a.y - v.y};
            *p0 = C{a.x + v.x, a.y + v.y};
            *p1 = C{w.x * d.x - w.y * d.y, w.x * d.y + w.y * d.x};
        }
        __syncthreads();
    }
}

constexpr int kFftLdsBytes = 49152;   // LDS per workgroup for one batch
constexpr int kFftThreads = 256;

// ---------------------------------------------------------------- x pass
// batch of RB rows (c, z, y); forward: keep modes 0..K
template <typename R>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_fwd(int logn, int nrows, int K1,
                                                         const R *__restrict__ grid,
                                                         const typename Cx<R>::T *__restrict__ tw,
                                                         typename Cx<R>::T *__restrict__ A) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    C *buf = (C *)smem;
    const int n = 1 << logn, RB = kFftLdsBytes / (int)sizeof(C) / n;
    const int row0 = blockIdx.x * RB;
    const int nr = nrows - row0 < RB ? nrows - row0 : RB;
    for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
        const int r = i >> logn, j = i & (n - 1);
        const R v = r < nr ? grid[(size_t)(row0 + r) * n + j] : (R)0;
        buf[bitrev(j, logn) * RB + r] = C{v, (R)0};
    }
    __syncthreads();
    fft_dit(buf, logn, RB, tw);
    for (int i = threadIdx.x; i < nr * K1; i += blockDim.x) {
        const int r = i / K1, m = i - r * K1;
        A[(size_t)(row0 + r) * K1 + m] = buf[m * RB + r];
    }
}

// inverse: modes 0..K of each row, Hermitian completion, real part out
template <typename R>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_inv(int logn, int nrows, int K1,
                                                         const typename Cx<R>::T *__restrict__ A,
                                                         const typename Cx<R>::T *__restrict__ tw,
                                                         R *__restrict__ grid) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    C *buf = (C *)smem;
    const int n = 1 << logn, RB = kFftLdsBytes / (int)sizeof(C) / n;
    const int row0 = blockIdx.x * RB;
    const int nr = nrows - row0 < RB ? nrows - row0 : RB;
    for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
        const int r = i % RB, m = i / RB;
        C v = C{(R)0, (R)0};
        if (r < nr) {
            if (m < K1) v = A[(size_t)(row0 + r) * K1 + m];
            else if (n - m < K1) {
                const C u = A[(size_t)(row0 + r) * K1 + (n - m)];
                v = C{u.x, -u.y};
            }
        }
        buf[i] = v;
    }
    __syncthreads();
    fft_dif(buf, logn, RB, tw);
    for (int i = threadIdx.x; i < nr * n; i += blockDim.x) {
        const int r = i >> logn, j = i & (n - 1);
        grid[(size_t)(row0 + r) * n + j] = buf[bitrev(j, logn) * RB + r].x;
    }
}

// ---------------------------------------------------------------- y pass
// one workgroup per (c, z) and group of KB columns mx
template <typename R>
__global__ __launch_bounds__(kFftThreads) void k_fft_y_fwd(int logn, int K, int KB,
                                                         const typename Cx<R>::T *__restrict__ A,
                                                         const typename Cx<R>::T *__restrict__ tw,
                                                         typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    C *buf = (C *)smem;
    const int n = 1 << logn, K1 = K + 1, NY = 2 * K + 1;
    const int ngrp = (K1 + KB - 1) / KB;
    const int g = blockIdx.x % ngrp, cz = blockIdx.x / ngrp;   // cz = c * n + z
    const int c = cz >> logn, z = cz & (n - 1);
    const int kx0 = g * KB;
    for (int i = threadIdx.x; i < n * KB; i += blockDim.x) {
        const int y = i / KB, q = i - y * KB;
        const int kx = kx0 + q;
        buf[bitrev(y, logn) * KB + q] =
            kx < K1 ? A[((size_t)cz * n + y) * K1 + kx] : C{(R)0, (R)0};
    }
    __syncthreads();
    fft_dit(buf, logn, KB, tw);
    for (int i = threadIdx.x; i < NY * KB; i += blockDim.x) {
        const int myp = i / KB, q = i - myp * KB;
        const int kx = kx0 + q;
        if (kx >= K1) continue;
        int y = myp - K;
        if (y < 0) y += n;
        B[(((size_t)c * NY + myp) * n + z) * K1 + kx] = buf[y * KB + q];
    }
}

template <typename R>
__global__ __launch_bounds__(kFftThreads) void k_fft_y_inv(int logn, int K, int KB,
                                                         const typename Cx<R>::T *__restrict__ B,
                                                         const typename Cx<R>::T *__restrict__ tw,
                                                         typename Cx<R>::T *__restrict__ A) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    C *buf = (C *)smem;
    const int n = 1 << logn, K1 = K + 1, NY = 2 * K + 1;
    const int ngrp = (K1 + KB - 1) / KB;
    const int g = blockIdx.x % ngrp, cz = blockIdx.x / ngrp;
    const int c = cz >> logn, z = cz & (n - 1);
    const int kx0 = g * KB;
    for (int i = threadIdx.x; i < n * KB; i += blockDim.x) {
        const int y = i / KB, q = i - y * KB;
        const int kx = kx0 + q;
        const int my = y <= n / 2 ? y : y - n;
        C v = C{(R)0, (R)0};
        if (kx < K1 && my >= -K && my <= K)
            v = B[(((size_t)c * NY + (my + K)) * n + z) * K1 + kx];
        buf[i] = v;
    }
    __syncthreads();
    fft_dif(buf, logn, KB, tw);
    for (int i = threadIdx.x; i < n * KB; i += blockDim.x) {
        const int y = i / KB, q = i - y * KB;
        const int kx = kx0 + q;
        if (kx < K1) A[((size_t)cz * n + y) * K1 + kx] = buf[bitrev(y, logn) * KB + q];
    }
}

// ---------------------------------------------------------------- z pass
// one workgroup per (my, group of KZ columns mx): the three components'
// z-columns, forward FFT, spectral operator, inverse FFT, written back.
// Sequence s = c * KZ + q; element mz of it at buf[mz * 3KZ + s].
template <typename R>
__global__ __launch_bounds__(kFftThreads) void k_fft_z_spectral(
    int logn, int K, int KZ, int psi, double k0, double inv4a2, double invV,
    const double *__restrict__ dec2, const typename Cx<R>::T *__restrict__ twf,
    const typename Cx<R>::T *__restrict__ twi, typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    C *buf = (C *)smem;
    const int n = 1 << logn, K1 = K + 1, NY = 2 * K + 1, S = 3 * KZ;
    const int ngrp = (K1 + KZ - 1) / KZ;
    const int g = blockIdx.x % ngrp, myp = blockIdx.x / ngrp;
    const int kx0 = g * KZ;
    const size_t cstride = (size_t)NY * n * K1;
    for (int i = threadIdx.x; i < n * S; i += blockDim.x) {
        const int z = i / S, s = i - z * S;
        const int c = s / KZ, q = s - c * KZ;
        const int kx = kx0 + q;
        buf[bitrev(z, logn) * S + s] =
            kx < K1 ? B[c * cstride + ((size_t)myp * n + z) * K1 + kx] : C{(R)0, (R)0};
    }
    __syncthreads();
    fft_dit(buf, logn, S, twf);
    const int my = myp - K;
    for (int i = threadIdx.x; i < n * KZ; i += blockDim.x) {
        const int z = i / KZ, q = i - z * KZ;
        const int mx = kx0 + q, mz = z <= n / 2 ? z : z - n;
        C *G0 = buf + z * S + q, *G1 = G0 + KZ, *G2 = G1 + KZ;
        const int ay = my < 0 ? -my : my, az = mz < 0 ? -mz : mz;
        if (mx >= K1 || az > K || (mx == 0 && my == 0 && mz == 0)) {
            *G0 = *G1 = *G2 = C{(R)0, (R)0};
            continue;
        }
        const double kx = k0 * mx, ky = k0 * my, kz = k0 * mz;
        const double k2 = kx * kx + ky * ky + kz * kz;
        const double f = exp(-k2 * inv4a2) / k2 * invV * dec2[mx] * dec2[ay] * dec2[az];
        const C g0 = *G0, g1 = *G1, g2 = *G2;
        if (psi) {
            const R fr = (R)f;
            *G0 = C{g0.x * fr, g0.y * fr};
            *G1 = C{g1.x * fr, g1.y * fr};
            *G2 = C{g2.x * fr, g2.y * fr};
            continue;
        }
        // i (k x G) f
        const R fkx = (R)(kx * f), fky = (R)(ky * f), fkz = (R)(kz * f);
        const R cr0 = fky * g2.x - fkz * g1.x, ci0 = fky * g2.y - fkz * g1.y;
        const R cr1 = fkz * g0.x - fkx * g2.x, ci1 = fkz * g0.y - fkx * g2.y;
        const R cr2 = fkx * g1.x - fky * g0.x, ci2 = fkx * g1.y - fky * g0.y;
        *G0 = C{-ci0, cr0};
        *G1 = C{-ci1, cr1};
        *G2 = C{-ci2, cr2};
    }
    __syncthreads();
    fft_dif(buf, logn, S, twi);
    for (int i = threadIdx.x; i < n * S; i += blockDim.x) {
        const int z = i / S, s = i - z * S;
        const int c = s / KZ, q = s - c * KZ;
        const int kx = kx0 + q;
        if (kx < K1) B[c * cstride + ((size_t)myp * n + z) * K1 + kx] = buf[bitrev(z, logn) * S + s];
    }
}

// --------------------------------------------------------------- launch
bool pruned_fft_ok(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

static int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) l++;
    return l;
}

template <typename R>
static void pruned_fwd(bs_plan_t p) {
    typedef typename Cx<R>::T C;
    const int n = p->n, logn = ilog2(n), K = p->prm.K, K1 = K + 1;
    const int nrows = 3 * n * n;
    const int RB = kFftLdsBytes / (int)sizeof(C) / n;
    const C *twf = (const C *)p->fft_tw.p;
    hipLaunchKernelGGL(k_fft_x_fwd<R>, dim3(ceil_div(nrows, RB)), dim3(kFftThreads),
                       RB * n * sizeof(C), p->stream, logn, nrows, K1, (const R *)p->grid.p, twf,
                       (C *)p->fft_A.p);
    const int KB = p->fft_kb;
    const int ngrp = ceil_div(K1, KB);
    hipLaunchKernelGGL(k_fft_y_fwd<R>, dim3(3 * n * ngrp), dim3(kFftThreads), n * KB * sizeof(C),
                       p->stream, logn, K, KB, (const C *)p->fft_A.p, twf, (C *)p->fft_B.p);
}

template <typename R>
static void pruned_spectral(bs_plan_t p, int psi) {
    typedef typename Cx<R>::T C;
    const int n = p->n, logn = ilog2(n), K = p->prm.K, K1 = K + 1, KZ = p->fft_kz;
    const double L = p->prm.L;
    const double k0 = 2.0 * kPi / L, inv4a2 = 1.0 / (4.0 * p->prm.alpha * p->prm.alpha);
    const double *dec2 = (const double *)p->deconv.p + (p->prm.K + 1);
    const C *twf = (const C *)p->fft_tw.p, *twi = twf + n / 2;
    hipLaunchKernelGGL(k_fft_z_spectral<R>, dim3((2 * K + 1) * ceil_div(K1, KZ)),
                       dim3(kFftThreads), 3 * n * KZ * sizeof(C), p->stream, logn, K, KZ, psi, k0,
                       inv4a2, 1.0 / (L * L * L), dec2, twf, twi, (C *)p->fft_B.p);
}

template <typename R>
static void pruned_inv(bs_plan_t p) {
    typedef typename Cx<R>::T C;
    const int n = p->n, logn = ilog2(n), K = p->prm.K, K1 = K + 1;
    const int nrows = 3 * n * n;
    const int RB = kFftLdsBytes / (int)sizeof(C) / n;
    const C *twi = (const C *)p->fft_tw.p + n / 2;
    const int KB = p->fft_kb;
    const int ngrp = ceil_div(K1, KB);
    hipLaunchKernelGGL(k_fft_y_inv<R>, dim3(3 * n * ngrp), dim3(kFftThreads), n * KB * sizeof(C),
                       p->stream, logn, K, KB, (const C *)p->fft_B.p, twi, (C *)p->fft_A.p);
    hipLaunchKernelGGL(k_fft_x_inv<R>, dim3(ceil_div(nrows, RB)), dim3(kFftThreads),
                       RB * n * sizeof(C), p->stream, logn, nrows, K1, (const C *)p->fft_A.p, twi,
                       (R *)p->grid.p);
}

void pruned_forward(bs_plan_t p) {
    if (p->fp32) pruned_fwd<float>(p); else pruned_fwd<double>(p);
}
void pruned_spectral_op(bs_plan_t p, int psi) {
    if (p->fp32) pruned_spectral<float>(p, psi); else pruned_spectral<double>(p, psi);
}
void pruned_inverse(bs_plan_t p) {
    if (p->fp32) pruned_inv<float>(p); else pruned_inv<double>(p);
}

// batch sizes: columns per workgroup in the y pass (KB) and z pass (KZ), so
// that one batch fills at most kFftLdsBytes of LDS
void pruned_batches(int n, size_t csize, int *kb, int *kz) {
    int b = (int)(kFftLdsBytes / (csize * n));
    int z = (int)(kFftLdsBytes / (3 * csize * n));
    *kb = b < 1 ? 1 : (b > 16 ? 16 : b);
    *kz = z < 1 ? 1 : (z > 16 ? 16 : z);
}

}  // namespace bs
