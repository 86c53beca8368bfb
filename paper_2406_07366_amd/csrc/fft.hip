// Pruned 3-D transforms of the long-range step (Sec. 3.3) for power-of-two
// grids: only the retained modes |m_i| <= K (K < n/2) are ever formed or
// stored past the first transform of each direction, and the spectral
// operator is applied between the forward and inverse z transforms of the
// same columns, so it costs no pass of its own.
//
//   x forward   grid [3][n][n][n] real (x fastest), rows r = (c n + z) n + y
//               ->  A [0..K][3 n^2]: mode kx of every row, rows fastest
//   y forward   A, FFT along y (sequence q = (3 kx + c) n + z is contiguous),
//               keep my in [-K, K]   ->  B [my+K][0..K][3][n] (z fastest)
//   z fused     B, FFT along z (contiguous), spectral operator (modes with
//               |mz| > K, k = 0 zeroed), inverse FFT along z  ->  B in place
//   y inverse   B, zero-padded inverse FFT along y  ->  A
//   x inverse   A, Hermitian c2r along x  ->  grid with the three components
//               interleaved, [n][n][n][3] (the interpolation's layout; the
//               spread writes [3][n][n][n])
//
// Every pass reads or writes whole contiguous sequences on one side; on the
// other it moves 128-B runs (16 float32 or 8 float64 complex values of
// neighbouring rows or z), which is why a workgroup takes that many
// sequences.  (On grids up to 64^3 the x and y passes are fused per plane
// and B is laid out [3][my+K][z][0..K]; see k_fft_xy_fwd.)
//
// Conventions are those of an unnormalised r2c / c2r pair: forward
// exp(-2 pi i j m / n), inverse exp(+2 pi i j m / n), no scaling (the
// spectral operator carries 1/L^3 and the deconvolution).
//
// Each workgroup transforms a batch of nseq sequences by a Stockham autosort
// FFT (natural order in and out): passes of radix 16, 8, 4 or 2 done in
// registers, one item per thread and pass, twiddle factors from a
// full-circle table.  The first pass reads its elements straight from global
// memory and the last writes straight to it; passes in between exchange
// through one LDS buffer with element j of sequence s at buf[j * pitch + s]
// (pitch = nseq + 1, odd, so strided accesses spread over the banks).  A
// 256-point transform (16 x 16) therefore touches LDS once each way.
#include <atomic>
#include <type_traits>

#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

template <typename R> struct Cx;
template <> struct Cx<float> { typedef float2 T; };
template <> struct Cx<double> { typedef double2 T; };

// cos and sin of 2 pi m / 16
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128676, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128676,
    -1.0, -0.92387953251128676, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128676};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128676,
    1.0, 0.92387953251128676, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128676,
    -1.0, -0.92387953251128676, -0.70710678118654752, -0.38268343236508977};

// In-register DFT of size R <= 16 (sgn -1 forward, +1 inverse): radix-2
// decimation in time with the bit reversal resolved at compile time.
template <int R, typename C, typename T>
__device__ __forceinline__ void dft_regs(C (&v)[R], T sgn) {
    constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : (R == 8 ? 3 : 4));
#pragma unroll
    for (int i = 0; i < R; i++) {
        int j = 0;
#pragma unroll
        for (int bb = 0; bb < LR; bb++)
            if (i & (1 << bb)) j |= 1 << (LR - 1 - bb);
        if (j > i) {
            const C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int half = 1; half < R; half <<= 1) {
#pragma unroll
        for (int k = 0; k < R; k += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; j++) {
                const int m = j * (8 / half);   // angle 2 pi j / (2 half) = 2 pi m / 16
                const T c = (T)kCos16[m], s = sgn * (T)kSin16[m];
                const C bq = v[k + j + half], a = v[k + j];
                const C t = C{c * bq.x - s * bq.y, c * bq.y + s * bq.x};
                v[k + j] = C{a.x + t.x, a.y + t.y};
                v[k + j + half] = C{a.x - t.x, a.y - t.y};
            }
        }
    }
}

// Radix plan of a length-2^logn transform: passes of radix at most 16,
// balanced (16 = 16, 32 = 8.4, 64 = 8.8, 128 = 16.8, 256 = 16.16,
// 512 = 8.8.8, 1024 = 16.8.8).  Returns the number of passes.
__host__ __device__ inline int fft_plan(int logn, int *lr) {
    int np = 0, rem = logn;
    while (rem > 0) {
        const int passes = (rem + 3) / 4;
        const int l = (rem + passes - 1) / passes;
        lr[np++] = l;
        rem -= l;
    }
    return np;
}

// items (threads) per sequence in the pass with the smallest radix
__host__ __device__ inline int fft_max_nj(int logn) {
    int lr[4];
    const int np = fft_plan(logn, lr);
    int mn = 4;
    for (int p = 0; p < np; p++) mn = lr[p] < mn ? lr[p] : mn;
    return (1 << logn) >> mn;
}

// One radix-R Stockham pass over nseq sequences of length n = nj R (Ns is
// the product of the radices of the passes before; tw[k] = exp(sgn 2 pi i
// k / n)).  Thread t owns item (s, j): s = t / nj, j = t % nj when JFAST
// (lanes along the sequence), else s = t % nseq, j = t / nseq (lanes across
// sequences).  It reads elements j + r nj (from load() in the first pass,
// else from LDS), applies the twiddles and an in-register DFT, and writes
// elements (j - j mod Ns) R + j mod Ns + r Ns (to store() in the last pass,
// else to LDS).  One LDS buffer: every read is done before any write.
// LDS position of element e of sequence s: lanes along a sequence (JFAST)
// use sequence-major rows skewed by one slot every 16 elements (the first
// pass writes 16 consecutive elements per thread, so lanes are 16 apart);
// lanes across sequences use element-major rows of pitch nseq + 1.
template <bool JFAST>
__device__ __forceinline__ int lds_at(int s, int e, int pitch) {
    return JFAST ? s * pitch + e + (e >> 4) : e * pitch + s;
}

template <bool JFAST>
__host__ __device__ inline int lds_pitch(int n, int nseq) {
    return JFAST ? n + (n >> 4) + 1 : nseq + 1;
}

// radix 2^lr of pass p of the plan above (0 past the last pass)
__host__ __device__ constexpr int plan_lr(int logn, int p) {
    int rem = logn;
    for (int q = 0; q <= p; q++) {
        if (rem <= 0) return 0;
        const int passes = (rem + 3) / 4, l = (rem + passes - 1) / passes;
        if (q == p) return l;
        rem -= l;
    }
    return 0;
}

// The transform length, the radix, Ns and whether the pass is the first
// or the last are compile-time, so the index arithmetic folds to shifts
// and masks and the pass sequence unrolls.  Each thread owns IPT items
// (t, t + blockDim, ...), all read before the barrier and written after it.
// The first pass applies no twiddles, so hook() (the twiddle table's own
// copy into LDS) runs after its loads are issued: one memory round trip for
// both.  TWCONJ: the table holds exp(-2 pi i k / n) and the pass uses its
// conjugates (an inverse transform from the forward table).
struct NoHook {
    __device__ void operator()() const {}
};

template <int R, int N, int NS, bool FIRST, bool LAST, bool JFAST, int IPT, bool TWCONJ,
          typename C, typename T, typename Load, typename Store, typename Hook>
__device__ __forceinline__ void fft_pass(int nseq, int pitch, C *buf, const C *tw, T sgn,
                                         Load &load, Store &store, Hook &hook) {
    constexpr int NJ = N / R;
    C v[IPT][R];
    int sv[IPT], jv[IPT];
    bool act[IPT];
#pragma unroll
    for (int it = 0; it < IPT; it++) {
        const int t = threadIdx.x + it * blockDim.x;
        act[it] = t < NJ * nseq;
        const int s = JFAST ? t / NJ : t % nseq, j = JFAST ? t % NJ : t / nseq;
        sv[it] = s;
        jv[it] = j;
        if (act[it]) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int e = j + r * NJ;
                if constexpr (FIRST) v[it][r] = load(s, e);
                else v[it][r] = buf[lds_at<JFAST>(s, e, pitch)];
            }
        }
    }
    if constexpr (FIRST) hook();
#pragma unroll
    for (int it = 0; it < IPT; it++) {
        if (act[it]) {
            if constexpr (NS > 1) {
                const int jm = jv[it] & (NS - 1);
                if (jm != 0) {
                    constexpr int STEP = N / (NS * R);
#pragma unroll
                    for (int r = 1; r < R; r++) {
                        const C w0 = tw[jm * r * STEP];
                        const C w = TWCONJ ? C{w0.x, -w0.y} : w0;
                        const C u = v[it][r];
                        v[it][r] = C{w.x * u.x - w.y * u.y, w.x * u.y + w.y * u.x};
                    }
                }
            }
            dft_regs<R>(v[it], sgn);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IPT; it++) {
        if (act[it]) {
            const int j = jv[it], jm = j & (NS - 1), d0 = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int e = d0 + r * NS;
                if constexpr (LAST) store(sv[it], e, v[it][r]);
                else buf[lds_at<JFAST>(sv[it], e, pitch)] = v[it][r];
            }
        }
    }
    __syncthreads();
}

// tw: the twiddle table in LDS (n entries); passes P, P+1, ... of the plan
template <bool JFAST, int LOGN, int IPT = 1, bool TWCONJ = false, int P = 0, int NS = 1,
          typename C, typename T, typename Load, typename Store, typename Hook>
__device__ __forceinline__ void fft_run_h(int nseq, int pitch, C *buf, const C *tw, T sgn,
                                          Load &load, Store &store, Hook &hook) {
    constexpr int LR = plan_lr(LOGN, P);
    if constexpr (LR > 0) {
        constexpr bool LAST = plan_lr(LOGN, P + 1) == 0;
        fft_pass<1 << LR, 1 << LOGN, NS, P == 0, LAST, JFAST, IPT, TWCONJ>(nseq, pitch, buf, tw,
                                                                           sgn, load, store, hook);
        fft_run_h<JFAST, LOGN, IPT, TWCONJ, P + 1, (NS << LR)>(nseq, pitch, buf, tw, sgn, load,
                                                               store, hook);
    }
}

template <bool JFAST, int LOGN, int IPT = 1, bool TWCONJ = false, typename C, typename T,
          typename Load, typename Store>
__device__ __forceinline__ void fft_run(int nseq, int pitch, C *buf, const C *tw, T sgn,
                                        Load &load, Store &store) {
    NoHook none;
    fft_run_h<JFAST, LOGN, IPT, TWCONJ>(nseq, pitch, buf, tw, sgn, load, store, none);
}

// copy ntab twiddle entries into LDS (before the first barrier of fft_run)
template <typename C>
__device__ __forceinline__ void stage_twiddles(C *dst, const C *__restrict__ src, int ntab) {
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) dst[i] = src[i];
}

// cnt items into LDS: store(i, load(i)), with up to B loads of each thread in
// flight before their LDS stores (a plain loop would wait for every load)
template <int B, typename Load, typename Store>
__device__ __forceinline__ void gather_lds(int cnt, Load &load, Store &store) {
    for (int i0 = threadIdx.x; i0 < cnt; i0 += B * blockDim.x) {
        decltype(load(0)) v[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const int i = i0 + b * (int)blockDim.x;
            if (i < cnt) v[b] = load(i);
        }
#pragma unroll
        for (int b = 0; b < B; b++) {
            const int i = i0 + b * (int)blockDim.x;
            if (i < cnt) store(i, v[b]);
        }
    }
}

constexpr int kFftMaxThreads = 512;
constexpr int kFftLds = 65536;        // LDS per workgroup, at most (x, y passes)
constexpr int kFftLdsZ = 81920;       // z pass with several items per thread (two
                                      // workgroups per CU; measured faster than one)

// items per thread of the z pass: large float32 grids take several columns
// per thread so that a workgroup spans enough adjacent columns mx for its
// loads and stores to coalesce (measured slower in float64, where the LDS
// then allows one workgroup per CU)
__host__ __device__ constexpr int z_ipt(int logn, int csize) {
    return logn >= 9 && csize == 8 ? 4 : 1;
}

// -------------------------------------------- large grids (n >= 128)
// Sequences per workgroup: the 128-B run (16 float32 or 8 float64 complex
// values) of the transposed side; items per thread so that a workgroup has at
// most kFftMaxThreads threads.
template <typename C> __host__ __device__ constexpr int run_len() { return 128 / (int)sizeof(C); }
// rows per x-pass workgroup, sequences per y-pass workgroup (the inverse y
// pass measured faster at 8 sequences in float32 too: 64-B runs, half the LDS,
// twice the workgroups per CU: 1.23 -> 1.05 ms for the inverse at 512^3;
// the forward pass and the x passes slower that way)
template <typename C> __host__ __device__ constexpr int x_rows() { return run_len<C>(); }
template <typename C> __host__ __device__ constexpr int y_seqs() { return run_len<C>(); }
template <typename C> __host__ __device__ constexpr int y_inv_seqs() { return 8; }
__host__ __device__ constexpr int min_radix_log(int logn) {
    int m = 4;
    for (int p = 0; plan_lr(logn, p) > 0; p++) m = plan_lr(logn, p) < m ? plan_lr(logn, p) : m;
    return m;
}
__host__ __device__ constexpr int fft_ipt(int logn, int nseq) {
    const int items = nseq * ((1 << logn) >> min_radix_log(logn));
    return (items + kFftMaxThreads - 1) / kFftMaxThreads;   // rounded up
}
__host__ __device__ constexpr int fft_threads(int logn, int nseq) {
    const int items = nseq * ((1 << logn) >> min_radix_log(logn)), ipt = fft_ipt(logn, nseq);
    return (items + ipt - 1) / ipt;
}
// (my, mx) columns per z-pass workgroup (times 3 components): one, so that
// the LDS allows the most workgroups per CU (two measured 0.68 -> 0.88 ms in
// float64 and 0.32 -> 0.47 ms in float32 at 512^3)
template <typename C> __host__ __device__ constexpr int z_cols() { return 1; }

// x forward: run_len rows (consecutive y) per workgroup, two real rows per
// complex transform: sequence s carries rows a = row0 + 2 s and b = a + 1 as
// z = x_a + i x_b, and the spectra separate as X_a(k) = (Z(k) + conj Z(n-k))
// / 2, X_b(k) = (Z(k) - conj Z(n-k)) / (2i) for the kept modes k = 0..K.
// Mode k of the workgroup's rows goes to A[k][row0 ..] as one run.
template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_x_fwd(int nrows, int K1, int per,
                                                            const R *__restrict__ grid,
                                                            const typename Cx<R>::T *__restrict__ tw,
                                                            typename Cx<R>::T *__restrict__ A) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN, ROWS = x_rows<C>(), NSEQ = ROWS / 2;
    constexpr int IPT = fft_ipt(LOGN, NSEQ);
    C *twl = (C *)smem, *buf = twl + n;
    const int bid = xcd_block(per);
    if (bid >= nrows / ROWS) return;
    const size_t row0 = (size_t)bid * ROWS;
    const int pitch = lds_pitch<true>(n, NSEQ);
    auto load = [&](int s, int e) {
        return C{grid[(row0 + 2 * s) * n + e], grid[(row0 + 2 * s + 1) * n + e]};
    };
    // the spectrum Z stays in LDS (every read of the last pass precedes its
    // barrier, so its writes may go back into the same buffer)
    auto lstore = [&](int s, int e, C v) { buf[lds_at<true>(s, e, pitch)] = v; };
    auto hook = [&]() { stage_twiddles(twl, tw, n); };
    fft_run_h<true, LOGN, IPT>(NSEQ, pitch, buf, twl, (R)-1, load, lstore, hook);
#pragma unroll 4
    for (int i = threadIdx.x; i < ROWS * K1; i += blockDim.x) {
        const int r = i % ROWS, k = i / ROWS, sq = r >> 1;
        const C z = buf[lds_at<true>(sq, k, pitch)];
        const C zm = buf[lds_at<true>(sq, k == 0 ? 0 : n - k, pitch)];
        const R h = (R)0.5;
        A[(size_t)k * nrows + row0 + r] = (r & 1) ? C{h * (z.y + zm.y), h * (zm.x - z.x)}
                                                  : C{h * (z.x + zm.x), h * (z.y - zm.y)};
    }
}

// x inverse into the interpolation's layout: the grid leaves the inverse
// with its three components interleaved, g[((z n + y) n + x) 3 + c], so that
// a node's stencil row of three components is one contiguous run (the
// interpolation touches about half the cache lines it touches in [3][n]^3:
// 2.23 -> 1.63 ms in float64 at 512^3).  A workgroup takes the rows
// (z, y0 .. y0 + Y - 1) of all three components: the modes 0..K of each are
// gathered from A[k][(c n + z) n + y0 ..] (runs of Y) into LDS, and 3Y / 2
// complex transforms produce them, two real rows each: c0 + i c1 of row y,
// and c2 of rows y, y + 1 (both spectra Hermitian-completed).  Every (z, y)
// row's 3 n values are written by this workgroup alone.  The gathered
// spectra share the LDS of the transform's buffer: its first pass reads all
// of them before it writes.
template <typename C> __host__ __device__ constexpr int xi_rows() { return 64 / (int)sizeof(C); }

template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_x_inv(int K1, int per,
                                                            const typename Cx<R>::T *__restrict__ A,
                                                            const typename Cx<R>::T *__restrict__ tw,
                                                            R *__restrict__ grid) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN, Y = xi_rows<C>(), NSEQ = 3 * Y / 2;
    constexpr int IPT = fft_ipt(LOGN, NSEQ);
    constexpr size_t nrows = (size_t)3 * n * n;
    C *twl = (C *)smem, *buf = twl + n, *spec = buf;
    const int bid = xcd_block(per);
    if (bid >= n * (n / Y)) return;
    const int z = bid / (n / Y), y0 = (bid - z * (n / Y)) * Y;
    const int pitch = lds_pitch<true>(n, NSEQ);
    // the runs of modes 0..K (index i = (k 3 + c) Y + yy), then the twiddle
    // table, in one batched copy; spectrum of (c, yy) at spec[(c Y + yy) K1]
    const int nin = 3 * Y * K1;
    auto gl = [&](int i) {
        if (i >= nin) return tw[i - nin];
        const int yy = i % Y, kc = i / Y, c = kc % 3, k = kc / 3;
        return A[(size_t)k * nrows + ((size_t)c * n + z) * n + y0 + yy];
    };
    auto gs = [&](int i, C v) {
        if (i < nin) {
            const int yy = i % Y, kc = i / Y, c = kc % 3, k = kc / 3;
            spec[(c * Y + yy) * K1 + k] = v;
        } else {
            twl[i - nin] = v;
        }
    };
    gather_lds<8>(nin + n, gl, gs);
    __syncthreads();
    auto herm = [&](int c, int yy, int e) {
        const C *sp = spec + (c * Y + yy) * K1;
        C v = C{(R)0, (R)0};
        if (e < K1) v = sp[e];
        else if (n - e < K1) {
            const C u = sp[n - e];
            v = C{u.x, -u.y};
        }
        return v;
    };
    // sequence s < Y: components 0 and 1 of row y0 + s; s >= Y: component 2
    // of rows y0 + 2 (s - Y) and the next
    auto load = [&](int s, int e) {
        C a, b;
        if (s < Y) { a = herm(0, s, e); b = herm(1, s, e); }
        else { a = herm(2, 2 * (s - Y), e); b = herm(2, 2 * (s - Y) + 1, e); }
        return C{a.x - b.y, a.y + b.x};
    };
    // the last pass writes the real rows into LDS in the grid's interleaved
    // order (its barrier has retired every read of the buffer), and the
    // workgroup then copies its Y rows of 3 n values to the grid as one
    // contiguous block in 16-B stores (the block fits the transform's buffer)
    R *outl = (R *)buf;
    auto lstore = [&](int s, int e, C v) {
        if (s < Y) {
            R *g = outl + 3 * (s * n + e);
            g[0] = v.x;
            g[1] = v.y;
        } else {
            R *g = outl + 3 * ((2 * (s - Y)) * n + e) + 2;
            g[0] = v.x;
            g[3 * n] = v.y;
        }
    };
    fft_run<true, LOGN, IPT>(NSEQ, pitch, buf, twl, (R)1, load, lstore);
    typedef typename std::conditional<sizeof(R) == 8, double2, float4>::type V;
    constexpr int PER = 16 / (int)sizeof(R), NV = 3 * n * Y / PER;
    const V *src = (const V *)outl;
    V *dst = (V *)(grid + (size_t)3 * n * ((size_t)z * n + y0));
    for (int i = threadIdx.x; i < NV; i += blockDim.x) dst[i] = src[i];
}

// y forward: run_len sequences q = (3 kx + c) n + z0 + s (contiguous in A);
// mode my of the workgroup's sequences goes to B[my + K][kx][c][z0 ..] as
// one run
template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_y_fwd(int K, int per,
                                                            const typename Cx<R>::T *__restrict__ A,
                                                            const typename Cx<R>::T *__restrict__ tw,
                                                            typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN, SEQ = y_seqs<C>();
    constexpr int IPT = fft_ipt(LOGN, SEQ);
    const int K1 = K + 1, NY = 2 * K + 1;
    C *twl = (C *)smem, *buf = twl + n;
    const int bid = xcd_block(per);
    if (bid >= 3 * n / SEQ * K1) return;
    const size_t q0 = (size_t)bid * SEQ;
    const int pitch = lds_pitch<true>(n, SEQ);
    auto load = [&](int s, int e) { return A[(q0 + s) * n + e]; };
    auto lstore = [&](int s, int e, C v) { buf[lds_at<true>(s, e, pitch)] = v; };
    auto hook = [&]() { stage_twiddles(twl, tw, n); };
    fft_run_h<true, LOGN, IPT>(SEQ, pitch, buf, twl, (R)-1, load, lstore, hook);
    const size_t kxc = q0 >> LOGN;   // 3 kx + c
    const int z0 = (int)(q0 & (n - 1));
#pragma unroll 4
    for (int i = threadIdx.x; i < SEQ * NY; i += blockDim.x) {
        const int s = i % SEQ, ky = i / SEQ, my = ky - K;
        B[((size_t)ky * 3 * K1 + kxc) * n + z0 + s] = buf[lds_at<true>(s, my < 0 ? my + n : my, pitch)];
    }
}

// y inverse: the B runs of run_len sequences into LDS (modes |my| > K zero),
// inverse FFT along y, whole sequences out to A
template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_y_inv(int K, int per,
                                                            const typename Cx<R>::T *__restrict__ B,
                                                            const typename Cx<R>::T *__restrict__ tw,
                                                            typename Cx<R>::T *__restrict__ A) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN, SEQ = y_inv_seqs<C>();
    constexpr int IPT = fft_ipt(LOGN, SEQ);
    const int K1 = K + 1;
    C *twl = (C *)smem, *buf = twl + n;
    const int bid = xcd_block(per);
    if (bid >= 3 * n / SEQ * K1) return;
    const size_t q0 = (size_t)bid * SEQ, kxc = q0 >> LOGN;
    const int z0 = (int)(q0 & (n - 1));
    const int pitch = lds_pitch<true>(n, SEQ);
    // the runs of modes |my| <= K (the rest zero), then the twiddle table, in
    // one batched copy
    const int nin = SEQ * n;
    auto gl = [&](int i) {
        C v = C{(R)0, (R)0};
        if (i < nin) {
            const int e = i / SEQ, my = e <= n / 2 ? e : e - n;
            if (my >= -K && my <= K) v = B[((size_t)(my + K) * 3 * K1 + kxc) * n + z0 + i % SEQ];
        } else {
            v = tw[i - nin];
        }
        return v;
    };
    auto gs = [&](int i, C v) {
        if (i < nin) buf[lds_at<true>(i % SEQ, i / SEQ, pitch)] = v;
        else twl[i - nin] = v;
    };
    gather_lds<8>(nin + n, gl, gs);
    __syncthreads();
    auto load = [&](int s, int e) { return buf[lds_at<true>(s, e, pitch)]; };
    auto store = [&](int s, int e, C v) { A[(q0 + s) * n + e] = v; };
    fft_run<true, LOGN, IPT>(SEQ, pitch, buf, twl, (R)1, load, store);
}

// z pass: z_cols (my, mx) columns per workgroup, their three components'
// z-sequences contiguous in B: forward FFT into LDS, spectral operator,
// inverse FFT from LDS, written back in place
template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_zt_spectral(
    int K, int per, int psi, double k0, double inv4a2, double invV,
    const double *__restrict__ dec2, const typename Cx<R>::T *__restrict__ twf,
    typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN, KZ = z_cols<C>(), S = 3 * KZ;
    constexpr int IPT = fft_ipt(LOGN, S);
    const int K1 = K + 1, ncol = (2 * K + 1) * K1;
    C *twl = (C *)smem, *buf = twl + n;   // forward table only
    const int bid = xcd_block(per), col0 = bid * KZ;
    if (col0 >= ncol) return;
    const int nseq = 3 * (ncol - col0 < KZ ? ncol - col0 : KZ);
    C *Bw = B + (size_t)col0 * 3 * n;
    const int pitch = lds_pitch<true>(n, S);
    auto gload = [&](int s, int e) {
        return s < nseq ? Bw[(size_t)s * n + e] : C{(R)0, (R)0};
    };
    auto lstore = [&](int s, int e, C v) { buf[lds_at<true>(s, e, pitch)] = v; };
    auto hook = [&]() { stage_twiddles(twl, twf, n); };
    fft_run_h<true, LOGN, IPT>(S, pitch, buf, twl, (R)-1, gload, lstore, hook);
    for (int i = threadIdx.x; i < KZ * n; i += blockDim.x) {
        const int kk = i >> LOGN, z = i & (n - 1), col = col0 + kk;
        if (col >= ncol) continue;
        const int ky = col / K1, mx = col - ky * K1, my = ky - K, mz = z <= n / 2 ? z : z - n;
        C *G0 = buf + lds_at<true>(3 * kk, z, pitch), *G1 = buf + lds_at<true>(3 * kk + 1, z, pitch),
          *G2 = buf + lds_at<true>(3 * kk + 2, z, pitch);
        const int ay = my < 0 ? -my : my, az = mz < 0 ? -mz : mz;
        if (az > K || (mx == 0 && my == 0 && mz == 0)) {
            *G0 = *G1 = *G2 = C{(R)0, (R)0};
            continue;
        }
        const double kx = k0 * mx, ky_ = k0 * my, kz = k0 * mz;
        const double k2 = kx * kx + ky_ * ky_ + kz * kz;
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
        const R fkx = (R)(kx * f), fky = (R)(ky_ * f), fkz = (R)(kz * f);
        const R cr0 = fky * g2.x - fkz * g1.x, ci0 = fky * g2.y - fkz * g1.y;
        const R cr1 = fkz * g0.x - fkx * g2.x, ci1 = fkz * g0.y - fkx * g2.y;
        const R cr2 = fkx * g1.x - fky * g0.x, ci2 = fkx * g1.y - fky * g0.y;
        *G0 = C{-ci0, cr0};
        *G1 = C{-ci1, cr1};
        *G2 = C{-ci2, cr2};
    }
    __syncthreads();
    auto lload = [&](int s, int e) { return buf[lds_at<true>(s, e, pitch)]; };
    auto gstore = [&](int s, int e, C v) {
        if (s < nseq) Bw[(size_t)s * n + e] = v;
    };
    // inverse from the forward table (conjugated twiddles)
    fft_run<true, LOGN, IPT, true>(S, pitch, buf, twl, (R)1, lload, gstore);
}

// ------------------------------------------- x and y passes fused (n <= 64)
// On small grids one workgroup takes a whole (c, z) plane: the x transforms
// of its n rows with modes 0..K kept in LDS, then the y transforms of those
// K + 1 columns (and the reverse for the inverse), so the plane needs one
// launch and no intermediate array in HBM.  A 64^2 plane in float64 needs
// 93 KB of LDS (one workgroup per CU; 192 workgroups).
constexpr int kFftXYMaxLogn = 6;

template <typename C>
__host__ __device__ constexpr size_t xy_lds(int n, int K1) {
    return ((size_t)n + (size_t)n * K1 + (size_t)n * (n + (n >> 4) + 1)) * sizeof(C);
}

template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_xy_fwd(int K, int per,
                                                             const R *__restrict__ grid,
                                                             const typename Cx<R>::T *__restrict__ tw,
                                                             typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN;
    const int K1 = K + 1, NY = 2 * K + 1;
    C *twl = (C *)smem, *P = twl + n, *buf = P + n * K1;   // P[y][kx]
    const int cz = xcd_block(per);   // c * n + z
    if (cz >= 3 * n) return;
    stage_twiddles(twl, tw, n);
    const int c = cz >> LOGN, z = cz & (n - 1);
    const R *plane = grid + (size_t)cz * n * n;
    auto xload = [&](int s, int e) { return C{plane[(size_t)s * n + e], (R)0}; };
    auto xstore = [&](int s, int e, C v) {
        if (e < K1) P[s * K1 + e] = v;
    };
    fft_run<true, LOGN>(n, lds_pitch<true>(n, n), buf, twl, (R)-1, xload, xstore);
    auto yload = [&](int s, int e) { return P[e * K1 + s]; };
    auto ystore = [&](int s, int e, C v) {
        const int my = e <= n / 2 ? e : e - n;
        if (my >= -K && my <= K) B[(((size_t)c * NY + (my + K)) * n + z) * K1 + s] = v;
    };
    fft_run<false, LOGN>(K1, lds_pitch<false>(n, K1), buf, twl, (R)-1, yload, ystore);
}

template <typename R, int LOGN>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_yx_inv(int K, int per,
                                                             const typename Cx<R>::T *__restrict__ B,
                                                             const typename Cx<R>::T *__restrict__ tw,
                                                             R *__restrict__ grid) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN;
    const int K1 = K + 1, NY = 2 * K + 1;
    C *twl = (C *)smem, *P = twl + n, *buf = P + n * K1;
    const int cz = xcd_block(per);
    if (cz >= 3 * n) return;
    stage_twiddles(twl, tw, n);
    const int c = cz >> LOGN, z = cz & (n - 1);
    auto yload = [&](int s, int e) {
        const int my = e <= n / 2 ? e : e - n;
        C v = C{(R)0, (R)0};
        if (my >= -K && my <= K) v = B[(((size_t)c * NY + (my + K)) * n + z) * K1 + s];
        return v;
    };
    auto ystore = [&](int s, int e, C v) { P[e * K1 + s] = v; };
    fft_run<false, LOGN>(K1, lds_pitch<false>(n, K1), buf, twl, (R)1, yload, ystore);
    R *plane = grid + (size_t)cz * n * n;
    auto xload = [&](int s, int e) {
        C v = C{(R)0, (R)0};
        if (e < K1) v = P[s * K1 + e];
        else if (n - e < K1) {
            const C u = P[s * K1 + (n - e)];
            v = C{u.x, -u.y};
        }
        return v;
    };
    auto xstore = [&](int s, int e, C v) { plane[(size_t)s * n + e] = v.x; };
    fft_run<true, LOGN>(n, lds_pitch<true>(n, n), buf, twl, (R)1, xload, xstore);
}

// ------------------------------------------------ z pass (n <= 64)
// one workgroup per (my, group of KZ columns mx) of the per-plane layout
// B [3][my+K][z][0..K]: the three components' z-columns (sequence
// s = c KZ + q), forward FFT into LDS, spectral operator, inverse FFT from
// LDS, written back.
template <typename R, int LOGN, int IPT>
__global__ __launch_bounds__(kFftMaxThreads) void k_fft_z_spectral(
    int K, int KZ, int per, int psi, double k0, double inv4a2, double invV,
    const double *__restrict__ dec2, const typename Cx<R>::T *__restrict__ twf,
    const typename Cx<R>::T *__restrict__ twi, typename Cx<R>::T *__restrict__ B) {
    typedef typename Cx<R>::T C;
    extern __shared__ unsigned char smem[];
    constexpr int n = 1 << LOGN;
    const int K1 = K + 1, NY = 2 * K + 1, S = 3 * KZ, pitch = S + 1;
    C *twl = (C *)smem, *buf = twl + 2 * n;
    const int ngrp = (K1 + KZ - 1) / KZ;
    const int bid = xcd_block(per);
    if (bid >= NY * ngrp) return;
    stage_twiddles(twl, twf, 2 * n);   // forward then inverse (contiguous in the plan)
    const int g = bid % ngrp, myp = bid / ngrp;
    const int kx0 = g * KZ;
    const size_t cstride = (size_t)NY * n * K1;
    auto gload = [&](int s, int e) {
        const int c = s / KZ, kx = kx0 + (s - c * KZ);
        return kx < K1 ? B[c * cstride + ((size_t)myp * n + e) * K1 + kx] : C{(R)0, (R)0};
    };
    auto lstore = [&](int s, int e, C v) { buf[e * pitch + s] = v; };
    fft_run<false, LOGN, IPT>(S, pitch, buf, twl, (R)-1, gload, lstore);
    const int my = myp - K;
    for (int i = threadIdx.x; i < n * KZ; i += blockDim.x) {
        const int z = i / KZ, q = i - z * KZ;
        const int mx = kx0 + q, mz = z <= n / 2 ? z : z - n;
        C *G0 = buf + z * pitch + q, *G1 = G0 + KZ, *G2 = G1 + KZ;
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
    auto lload = [&](int s, int e) { return buf[e * pitch + s]; };
    auto gstore = [&](int s, int e, C v) {
        const int c = s / KZ, kx = kx0 + (s - c * KZ);
        if (kx < K1) B[c * cstride + ((size_t)myp * n + e) * K1 + kx] = v;
    };
    fft_run<false, LOGN, IPT>(S, pitch, buf, twl + n, (R)1, lload, gstore);
}

// --------------------------------------------------------------- launch
// power of two, and the z pass's smallest batch (2 twiddle tables + 3
// columns + pad) fits LDS
bool pruned_fft_ok(int n, size_t csize) {
    return n >= 16 && n <= 1024 && (n & (n - 1)) == 0 && (size_t)n * 6 * csize < kFftLds &&
           (size_t)3 * fft_max_nj(__builtin_ctz((unsigned)n)) <= kFftMaxThreads;
}

static int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) l++;
    return l;
}

// Kernels with more than 64 KB of dynamic LDS need the limit raised; the
// call is slow next to a launch, so it is made once per kernel and device,
// to the hardware maximum (a permission, not an allocation: plans with
// different needs share it safely).
constexpr int kLdsHwMax = 163840;
template <auto FN>
static void allow_big_lds(int device) {
    static std::atomic<unsigned long long> done{0};
    const unsigned long long bit = 1ull << (device & 63);
    if (!(done.load(std::memory_order_acquire) & bit)) {
        (void)hipFuncSetAttribute((const void *)FN, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kLdsHwMax);
        done.fetch_or(bit, std::memory_order_acq_rel);
    }
}

// call f(std::integral_constant<int, logn>) for the grid sizes the pruned
// path accepts (16 .. 1024)
template <typename F>
static void with_logn(int logn, F f) {
    switch (logn) {
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 9: f(std::integral_constant<int, 9>{}); break;
        default: f(std::integral_constant<int, 10>{}); break;
    }
}

// LDS of a large-grid pass: ntw twiddles + nseq skewed sequences
template <typename C>
static size_t seq_lds(int n, int nseq, int ntw) {
    return ((size_t)ntw + (size_t)nseq * lds_pitch<true>(n, nseq)) * sizeof(C);
}

template <typename R, int LOGN>
static void pruned_fwd(bs_plan_t p) {
    typedef typename Cx<R>::T C;
    constexpr int n = 1 << LOGN;
    const int K = p->prm.K, K1 = K + 1, mnj = fft_max_nj(LOGN);
    const C *twf = (const C *)p->fft_tw.p;
    if constexpr (LOGN <= kFftXYMaxLogn) {
        const size_t lds = xy_lds<C>(n, K1);
        if (lds > 65536) allow_big_lds<k_fft_xy_fwd<R, LOGN>>(p->device);
        const int per = ceil_div(3 * n, 8);
        hipLaunchKernelGGL((k_fft_xy_fwd<R, LOGN>), dim3(8 * per), dim3(n * mnj), lds, p->stream,
                           K, per, (const R *)p->grid.p, twf, (C *)p->fft_B.p);
    } else {
        constexpr int XR = x_rows<C>(), YS = y_seqs<C>();
        static_assert(fft_threads(LOGN, XR / 2) <= kFftMaxThreads &&
                          fft_threads(LOGN, YS) <= kFftMaxThreads,
                      "workgroups within the kernels' launch bounds");
        const int nrows = 3 * n * n;
        const int px = ceil_div(nrows / XR, 8), py = ceil_div(3 * n / YS * K1, 8);
        const size_t lx = seq_lds<C>(n, XR / 2, n), ly = seq_lds<C>(n, YS, n);
        if (lx > 65536) allow_big_lds<k_fft_x_fwd<R, LOGN>>(p->device);
        if (ly > 65536) allow_big_lds<k_fft_y_fwd<R, LOGN>>(p->device);
        hipLaunchKernelGGL((k_fft_x_fwd<R, LOGN>), dim3(8 * px), dim3(fft_threads(LOGN, XR / 2)),
                           lx, p->stream, nrows, K1, px, (const R *)p->grid.p, twf,
                           (C *)p->fft_A.p);
        hipLaunchKernelGGL((k_fft_y_fwd<R, LOGN>), dim3(8 * py), dim3(fft_threads(LOGN, YS)), ly,
                           p->stream, K, py, (const C *)p->fft_A.p, twf, (C *)p->fft_B.p);
    }
}

template <typename R, int LOGN>
static void pruned_spectral(bs_plan_t p, int psi) {
    typedef typename Cx<R>::T C;
    constexpr int n = 1 << LOGN;
    const int K = p->prm.K, K1 = K + 1;
    const double L = p->prm.L;
    const double k0 = 2.0 * kPi / L, inv4a2 = 1.0 / (4.0 * p->prm.alpha * p->prm.alpha);
    const double *dec2 = (const double *)p->deconv.p + (p->prm.K + 1);
    const C *twf = (const C *)p->fft_tw.p, *twi = twf + n;
    if constexpr (LOGN <= kFftXYMaxLogn) {
        const int KZ = p->fft_kz;
        const int pz = ceil_div((2 * K + 1) * ceil_div(K1, KZ), 8);
        constexpr int IPT = z_ipt(LOGN, (int)sizeof(C));
        const size_t lds = (2 * n + n * (3 * KZ + 1)) * sizeof(C);
        if (lds > 65536) allow_big_lds<k_fft_z_spectral<R, LOGN, IPT>>(p->device);
        hipLaunchKernelGGL((k_fft_z_spectral<R, LOGN, IPT>), dim3(8 * pz),
                           dim3(ceil_div(3 * KZ * fft_max_nj(LOGN), IPT)), lds, p->stream, K, KZ,
                           pz, psi, k0, inv4a2, 1.0 / (L * L * L), dec2, twf, twi,
                           (C *)p->fft_B.p);
    } else {
        constexpr int KZ = z_cols<C>();
        static_assert(fft_threads(LOGN, 3 * KZ) <= kFftMaxThreads,
                      "workgroups within the kernel's launch bounds");
        const int pz = ceil_div(ceil_div((2 * K + 1) * K1, KZ), 8);
        const size_t lds = seq_lds<C>(n, 3 * KZ, n);
        if (lds > 65536) allow_big_lds<k_fft_zt_spectral<R, LOGN>>(p->device);
        hipLaunchKernelGGL((k_fft_zt_spectral<R, LOGN>), dim3(8 * pz),
                           dim3(fft_threads(LOGN, 3 * KZ)), lds, p->stream, K, pz, psi, k0, inv4a2,
                           1.0 / (L * L * L), dec2, twf, (C *)p->fft_B.p);
    }
}

template <typename R, int LOGN>
static void pruned_inv(bs_plan_t p) {
    typedef typename Cx<R>::T C;
    constexpr int n = 1 << LOGN;
    const int K = p->prm.K, K1 = K + 1, mnj = fft_max_nj(LOGN);
    const C *twi = (const C *)p->fft_tw.p + n;
    if constexpr (LOGN <= kFftXYMaxLogn) {
        const size_t lds = xy_lds<C>(n, K1);
        if (lds > 65536) allow_big_lds<k_fft_yx_inv<R, LOGN>>(p->device);
        const int per = ceil_div(3 * n, 8);
        hipLaunchKernelGGL((k_fft_yx_inv<R, LOGN>), dim3(8 * per), dim3(n * mnj), lds, p->stream,
                           K, per, (const C *)p->fft_B.p, twi, (R *)p->grid.p);
    } else {
        constexpr int YS = y_inv_seqs<C>(), XY = xi_rows<C>(), XS = 3 * XY / 2;
        static_assert(fft_threads(LOGN, YS) <= kFftMaxThreads &&
                          fft_threads(LOGN, XS) <= kFftMaxThreads,
                      "workgroups within the kernels' launch bounds");
        const int px = ceil_div(n * (n / XY), 8), py = ceil_div(3 * n / YS * K1, 8);
        const size_t ly = seq_lds<C>(n, YS, n), lx = seq_lds<C>(n, XS, n);
        if (ly > 65536) allow_big_lds<k_fft_y_inv<R, LOGN>>(p->device);
        if (lx > 65536) allow_big_lds<k_fft_x_inv<R, LOGN>>(p->device);
        hipLaunchKernelGGL((k_fft_y_inv<R, LOGN>), dim3(8 * py), dim3(fft_threads(LOGN, YS)), ly,
                           p->stream, K, py, (const C *)p->fft_B.p, twi, (C *)p->fft_A.p);
        hipLaunchKernelGGL((k_fft_x_inv<R, LOGN>), dim3(8 * px), dim3(fft_threads(LOGN, XS)),
                           lx, p->stream, K1, px, (const C *)p->fft_A.p, twi, (R *)p->grid.p);
    }
}

bool grid_interleaved(bs_plan_t p) { return p->pruned && p->n > (1 << kFftXYMaxLogn); }

void pruned_forward(bs_plan_t p) {
    with_logn(ilog2(p->n), [&](auto L) {
        if (p->fp32) pruned_fwd<float, decltype(L)::value>(p);
        else pruned_fwd<double, decltype(L)::value>(p);
    });
}
void pruned_spectral_op(bs_plan_t p, int psi) {
    with_logn(ilog2(p->n), [&](auto L) {
        if (p->fp32) pruned_spectral<float, decltype(L)::value>(p, psi);
        else pruned_spectral<double, decltype(L)::value>(p, psi);
    });
}
void pruned_inverse(bs_plan_t p) {
    with_logn(ilog2(p->n), [&](auto L) {
        if (p->fp32) pruned_inv<float, decltype(L)::value>(p);
        else pruned_inv<double, decltype(L)::value>(p);
    });
}

// Batch sizes: sequences per workgroup for the x and y passes (rb = kb, a
// power of two) and columns for the z pass (kz, times 3 components): about
// 256 threads of one item each (128 in float64), with the LDS buffer and its
// padded pitch within kFftLds.
static int pow2_floor(int v) {
    int p = 1;
    while (2 * p <= v) p *= 2;
    return p;
}

void pruned_batches(int n, size_t csize, int *rb, int *kb, int *kz) {
    const int logn = ilog2(n), mnj = fft_max_nj(logn), ipt = z_ipt(logn, (int)csize);
    const int threads = csize > 8 ? 128 : 256;
    int b = threads / mnj;
    // twiddles (n, 2n in the z pass) + rows of about n + n/16 + 1 entries
    const int lds = (int)(kFftLds / (csize * (n + n / 16 + 1))) - 2;
    b = b < lds ? b : lds;
    b = pow2_floor(b < 1 ? 1 : b);
    *rb = b;
    *kb = b;
    // z pass: 3 kz sequences of mnj items, ipt items per thread, at most
    // kFftMaxThreads threads; LDS 2 twiddle tables + 3 kz + 1 columns
    const size_t zlds = ipt > 1 ? kFftLdsZ : kFftLds;
    int z = ipt > 1 ? kFftMaxThreads * ipt / (3 * mnj) : b / 3;
    z = z < 1 ? 1 : z;
    while (z > 1 && ((size_t)(2 * n + n * (3 * z + 1)) * csize > zlds ||
                     ceil_div(3 * z * mnj, ipt) > kFftMaxThreads))
        z--;
    *kz = z;
}

}  // namespace bs
