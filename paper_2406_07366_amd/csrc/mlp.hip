// Small MLP 8 -> 64 -> 64 -> 64 -> 3 (SiLU hidden activations) on BF16 MFMA
// with FP32 accumulation: inference, loss gradient and Adam training.  Used
// by the learned near-singular correction (no counterpart in the paper).  A
// debug mode (bs_mlp_set_fp32) runs the same kernels with FP32 weights and
// activations on FP32 MFMA, leaving only FP32 rounding in the gradients.
//
// Master parameters are FP32, packed W1[64][8] b1[64] W2[64][64] b2[64]
// W3[64][64] b3[64] W4[3][64] b4[3] (9091 values).  The kernels read a padded
// BF16 image of the weights:
//   W1p[64][16]: columns 0..7 and 8..15 both hold W1, so that the input
//                vector can be fed as (hi, lo) BF16 halves of each FP32
//                feature: W1 x = W1 hi + W1 lo keeps ~16 mantissa bits of x;
//   W2[64][64], W3[64][64];  W4p[16][64]: rows 3..15 zero;
// and FP32 biases b1, b2, b3 and b4p[16].
//
// One wavefront handles 16 samples at a time with v_mfma_f32_16x16x16_bf16
// in the transposed orientation Z^T = W H^T: the MFMA result layout (lane l
// holds rows 4(l/16)..4(l/16)+3 of column l%16) is exactly the B-operand
// layout of the next layer, so activations never leave registers in the
// forward pass.  Backward: dH^T = W^T dZ^T by MFMA in the same orientation;
// dW = dZ^T H by MFMA after a transpose of both 16-sample tiles through LDS.
// Weight gradients are summed per workgroup (one wavefront, plain adds) and
// the workgroup partials are added in a fixed order by a second kernel.
#include "bs_internal.h"

namespace bs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 64;                       // hidden width
constexpr int kNP = 9091;                    // master parameter count
// padded image offsets (in elements)
constexpr int kW1p = 0, kW2 = kW1p + 64 * 16, kW3 = kW2 + 64 * 64, kW4p = kW3 + 64 * 64;
constexpr int kWpad = kW4p + 16 * 64;        // 10240 bf16 weights
constexpr int kB1 = 0, kB2 = 64, kB3 = 128, kB4p = 192, kBpad = 208;   // fp32 biases
constexpr int kGpad = kWpad + kBpad;         // padded gradient length (fp32)

__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);          // round to nearest even
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
    return __uint_as_float(((unsigned int)h) << 16);
}
// SiLU and its derivative with the hardware exp2 and reciprocal (1 ulp in
// float32; the activations are rounded to bf16 right after)
__device__ __forceinline__ float sigmoid_f(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

// Precision of a kernel instance: F = false, BF16 operands on
// v_mfma_f32_16x16x16_bf16 (the product); F = true, FP32 weights and
// activations on v_mfma_f32_16x16x4_f32, four per 16x16x16 product (a debug
// mode that leaves only FP32 rounding, for checking the gradients tightly).
// The operand registers hold the same k indices in both: lane l, element j
// is k = 4(l/16) + j; the j-th FP32 MFMA sums k = j, 4 + j, 8 + j, 12 + j.
template <bool F> struct Prec {
    typedef unsigned short W;   // stored weights and tiles
    typedef bf16x4 Op;          // MFMA operand
    static __device__ __forceinline__ W store(float v) { return f2bf(v); }
    static __device__ __forceinline__ float elem(W w) { return bf2f(w); }
    static __device__ __forceinline__ f32x4 mfma(Op a, Op b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void set(Op &o, int r, W w) { o[r] = (short)w; }
};
template <> struct Prec<true> {
    typedef float W;
    typedef f32x4 Op;
    static __device__ __forceinline__ W store(float v) { return v; }
    static __device__ __forceinline__ float elem(W w) { return w; }
    static __device__ __forceinline__ f32x4 mfma(Op a, Op b, f32x4 c) {
#pragma unroll
        for (int j = 0; j < 4; j++) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
        return c;
    }
    static __device__ __forceinline__ void set(Op &o, int r, W w) { o[r] = w; }
};

template <bool F>
__device__ __forceinline__ f32x4 mfma16(typename Prec<F>::Op a, typename Prec<F>::Op b, f32x4 c) {
    return Prec<F>::mfma(a, b, c);
}

// A operand: 16x16 tile of a row-major matrix M (row stride ld), rows r0..,
// columns c0..: lane l reads M[r0 + l%16][c0 + 4(l/16) .. +3].
template <bool F>
__device__ __forceinline__ typename Prec<F>::Op load_a(const typename Prec<F>::W *M, int ld,
                                                       int r0, int c0, int l) {
    const typename Prec<F>::W *p = M + (r0 + (l & 15)) * ld + c0 + 4 * (l >> 4);
    typename Prec<F>::Op v;
    for (int r = 0; r < 4; r++) Prec<F>::set(v, r, p[r]);
    return v;
}
// A operand of the transpose: A[i][k] = M[k][i], i.e. lane l reads
// M[c0 + 4(l/16) + j][r0 + l%16], j = 0..3.
template <bool F>
__device__ __forceinline__ typename Prec<F>::Op load_at(const typename Prec<F>::W *M, int ld,
                                                        int r0, int c0, int l) {
    typename Prec<F>::Op v;
    int i = r0 + (l & 15), k = c0 + 4 * (l >> 4);
    for (int r = 0; r < 4; r++) Prec<F>::set(v, r, M[(k + r) * ld + i]);
    return v;
}
template <bool F>
__device__ __forceinline__ typename Prec<F>::Op to_op(f32x4 x) {
    typename Prec<F>::Op v;
    for (int r = 0; r < 4; r++) Prec<F>::set(v, r, Prec<F>::store(x[r]));
    return v;
}

template <bool F>
struct Fwd {
    f32x4 z1[4], z2[4], z3[4];   // pre-activations, blocks of 16 features
    typename Prec<F>::Op x;      // input operand (BF16: hi/lo halves; FP32: x, 0)
    f32x4 y;                     // outputs (rows 0..2 valid in lanes 0..15)
};

// input operand of the samples s0 .. s0+15: lanes 0..31 carry features 0..7,
// lanes 32..63 (the duplicated columns of W1p) the BF16 remainder x - hi, or
// zero in FP32
template <bool F>
__device__ __forceinline__ typename Prec<F>::Op input_op(const float *__restrict__ X, int64_t B,
                                                         int64_t s0, int l) {
    const int g = l >> 4;
    const int64_t s = s0 + (l & 15);
    float xv[4] = {0.f, 0.f, 0.f, 0.f};
    if (s < B) {
        const float *xs = X + 8 * s + 4 * (g & 1);
        for (int r = 0; r < 4; r++) {
            const float v = xs[r];
            if (F) {
                xv[r] = (g < 2) ? v : 0.f;
            } else {
                const float hi = bf2f(f2bf(v));
                xv[r] = (g < 2) ? hi : v - hi;
            }
        }
    }
    typename Prec<F>::Op x;
    for (int r = 0; r < 4; r++) Prec<F>::set(x, r, Prec<F>::store(xv[r]));
    return x;
}

// forward pass for samples s0 .. s0+15 (tail masked by B)
template <bool F>
__device__ __forceinline__ void mlp_tile_forward(const typename Prec<F>::W *W, const float *b,
                                                 const float *__restrict__ X, int64_t B,
                                                 int64_t s0, int l, Fwd<F> &f) {
    const int g = l >> 4;
    f.x = input_op<F>(X, B, s0, l);
    typename Prec<F>::Op h[4];
    for (int ob = 0; ob < 4; ob++) {
        f32x4 acc;
        for (int r = 0; r < 4; r++) acc[r] = b[kB1 + 16 * ob + 4 * g + r];
        acc = mfma16<F>(load_a<F>(W + kW1p, 16, 16 * ob, 0, l), f.x, acc);
        f.z1[ob] = acc;
    }
    for (int ob = 0; ob < 4; ob++) {
        f32x4 a = f.z1[ob];
        for (int r = 0; r < 4; r++) a[r] = silu(a[r]);
        h[ob] = to_op<F>(a);
    }
    for (int ob = 0; ob < 4; ob++) {
        f32x4 acc;
        for (int r = 0; r < 4; r++) acc[r] = b[kB2 + 16 * ob + 4 * g + r];
        for (int kb = 0; kb < 4; kb++) acc = mfma16<F>(load_a<F>(W + kW2, 64, 16 * ob, 16 * kb, l), h[kb], acc);
        f.z2[ob] = acc;
    }
    for (int ob = 0; ob < 4; ob++) {
        f32x4 a = f.z2[ob];
        for (int r = 0; r < 4; r++) a[r] = silu(a[r]);
        h[ob] = to_op<F>(a);
    }
    for (int ob = 0; ob < 4; ob++) {
        f32x4 acc;
        for (int r = 0; r < 4; r++) acc[r] = b[kB3 + 16 * ob + 4 * g + r];
        for (int kb = 0; kb < 4; kb++) acc = mfma16<F>(load_a<F>(W + kW3, 64, 16 * ob, 16 * kb, l), h[kb], acc);
        f.z3[ob] = acc;
    }
    for (int ob = 0; ob < 4; ob++) {
        f32x4 a = f.z3[ob];
        for (int r = 0; r < 4; r++) a[r] = silu(a[r]);
        h[ob] = to_op<F>(a);
    }
    f32x4 acc;
    for (int r = 0; r < 4; r++) acc[r] = b[kB4p + 4 * g + r];
    for (int kb = 0; kb < 4; kb++) acc = mfma16<F>(load_a<F>(W + kW4p, 64, 0, 16 * kb, l), h[kb], acc);
    f.y = acc;
}

template <typename WT>
__device__ void load_weights_lds(const WT *__restrict__ wg, const float *__restrict__ bg,
                                 WT *W, float *b) {
    for (int i = threadIdx.x; i < kWpad; i += blockDim.x) W[i] = wg[i];
    for (int i = threadIdx.x; i < kBpad; i += blockDim.x) b[i] = bg[i];
}

// ------------------------------------------------------------- inference
// The same arithmetic as mlp_tile_forward, with every weight operand and
// bias of the network held in registers across the wavefront's tiles (40
// A operands and 13 bias blocks, read from LDS once): a tile then costs its
// 40 MFMAs, 192 SiLUs per sample and the input and output accesses only.
template <bool F>
__global__ __launch_bounds__(256) void k_mlp_infer(int64_t B, const int *__restrict__ Bdev,
                                                   const float *__restrict__ X,
                                                   const typename Prec<F>::W *__restrict__ wg,
                                                   const float *__restrict__ bg,
                                                   float *__restrict__ Y) {
    typedef typename Prec<F>::Op Op;
    __shared__ typename Prec<F>::W W[kWpad];
    __shared__ float b[kBpad];
    if (Bdev) B = *Bdev;
    // a workgroup without a tile returns before staging the weights (the
    // launch is sized for the largest count; the device-side one is often
    // far smaller, or zero)
    if ((int64_t)blockIdx.x * (blockDim.x >> 6) >= (B + 15) / 16) return;
    load_weights_lds(wg, bg, W, b);
    __syncthreads();
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int g = l >> 4;
    Op A1[4], A2[4][4], A3[4][4], A4[4];
    f32x4 C1[4], C2[4], C3[4], C4;
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        A1[ob] = load_a<F>(W + kW1p, 16, 16 * ob, 0, l);
        A4[ob] = load_a<F>(W + kW4p, 64, 0, 16 * ob, l);
#pragma unroll
        for (int kb = 0; kb < 4; kb++) {
            A2[ob][kb] = load_a<F>(W + kW2, 64, 16 * ob, 16 * kb, l);
            A3[ob][kb] = load_a<F>(W + kW3, 64, 16 * ob, 16 * kb, l);
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            C1[ob][r] = b[kB1 + 16 * ob + 4 * g + r];
            C2[ob][r] = b[kB2 + 16 * ob + 4 * g + r];
            C3[ob][r] = b[kB3 + 16 * ob + 4 * g + r];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; r++) C4[r] = b[kB4p + 4 * g + r];
    const int64_t ntiles = (B + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * nw + wave; t < ntiles; t += (int64_t)gridDim.x * nw) {
        const int64_t s = 16 * t + (l & 15);
        const Op x = input_op<F>(X, B, 16 * t, l);
        Op h[4], hn[4];
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
            f32x4 a = mfma16<F>(A1[ob], x, C1[ob]);
#pragma unroll
            for (int r = 0; r < 4; r++) a[r] = silu(a[r]);
            h[ob] = to_op<F>(a);
        }
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
            f32x4 acc = C2[ob];
#pragma unroll
            for (int kb = 0; kb < 4; kb++) acc = mfma16<F>(A2[ob][kb], h[kb], acc);
#pragma unroll
            for (int r = 0; r < 4; r++) acc[r] = silu(acc[r]);
            hn[ob] = to_op<F>(acc);
        }
#pragma unroll
        for (int ob = 0; ob < 4; ob++) {
            f32x4 acc = C3[ob];
#pragma unroll
            for (int kb = 0; kb < 4; kb++) acc = mfma16<F>(A3[ob][kb], hn[kb], acc);
#pragma unroll
            for (int r = 0; r < 4; r++) acc[r] = silu(acc[r]);
            h[ob] = to_op<F>(acc);
        }
        f32x4 y = C4;
#pragma unroll
        for (int kb = 0; kb < 4; kb++) y = mfma16<F>(A4[kb], h[kb], y);
        if (g == 0 && s < B)
            for (int r = 0; r < 3; r++) Y[3 * s + r] = y[r];
    }
}

// ------------------------------------------------------------- training
// adds dZ^T H for one 16-sample tile into the LDS gradient accumulator G
// (out x in, row stride kin): Tz holds dZ [16][kout] and Th holds H [16][kin]
// in the instance's precision.
template <bool F>
__device__ __forceinline__ void acc_dw(const typename Prec<F>::W *Tz, int kout,
                                       const typename Prec<F>::W *Th, int kin, float *G, int l) {
    const int g = l >> 4;
    for (int ob = 0; ob < kout / 16; ob++)
        for (int ib = 0; ib < kin / 16; ib++) {
            typename Prec<F>::Op a, bb;
            for (int r = 0; r < 4; r++) {
                Prec<F>::set(a, r, Tz[(4 * g + r) * kout + 16 * ob + (l & 15)]);
                Prec<F>::set(bb, r, Th[(4 * g + r) * kin + 16 * ib + (l & 15)]);
            }
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = mfma16<F>(a, bb, d);
            for (int r = 0; r < 4; r++) G[(16 * ob + 4 * g + r) * kin + 16 * ib + (l & 15)] += d[r];
        }
}

// store a D-layout block (features 16*ob + 4g + r of sample l%16) into a
// [16][k] tile
template <bool F>
__device__ __forceinline__ void store_tile(typename Prec<F>::W *T, int k, int ob, f32x4 v, int l) {
    const int g = l >> 4;
    for (int r = 0; r < 4; r++) T[(l & 15) * k + 16 * ob + 4 * g + r] = Prec<F>::store(v[r]);
}

// bias gradient: sum over the 16 samples (lanes sharing l/16)
__device__ __forceinline__ void acc_db(f32x4 v, float *G, int base, int ob, int l) {
    for (int r = 0; r < 4; r++) {
        float s = v[r];
        for (int m = 1; m < 16; m <<= 1) s += __shfl_xor(s, m, 16);
        if ((l & 15) == 0) G[base + 16 * ob + 4 * (l >> 4) + r] += s;
    }
}

template <bool F>
__device__ __forceinline__ void hidden_back(const typename Prec<F>::W *W, float *G, int woff,
                                            int boff, const f32x4 (&zp)[4], f32x4 (&dz)[4],
                                            typename Prec<F>::W *Tz, typename Prec<F>::W *Th,
                                            bool valid, int l) {
    for (int ob = 0; ob < 4; ob++) {
        f32x4 h = zp[ob];
        for (int r = 0; r < 4; r++) h[r] = valid ? silu(h[r]) : 0.f;
        store_tile<F>(Th, 64, ob, h, l);
        store_tile<F>(Tz, 64, ob, dz[ob], l);
    }
    __syncthreads();
    acc_dw<F>(Tz, 64, Th, 64, G + woff, l);
    for (int ob = 0; ob < 4; ob++) acc_db(dz[ob], G, kWpad + boff, ob, l);
    __syncthreads();
    typename Prec<F>::Op dzb[4];
    for (int ob = 0; ob < 4; ob++) dzb[ob] = to_op<F>(dz[ob]);
    for (int ob = 0; ob < 4; ob++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kb = 0; kb < 4; kb++)
            acc = mfma16<F>(load_at<F>(W + woff, 64, 16 * ob, 16 * kb, l), dzb[kb], acc);
        for (int r = 0; r < 4; r++) acc[r] *= dsilu(zp[ob][r]);
        dz[ob] = acc;
    }
}

template <bool F>
__global__ __launch_bounds__(64) void k_mlp_train(int64_t B, const float *__restrict__ X,
                                                  const float *__restrict__ T, float scale,
                                                  const typename Prec<F>::W *__restrict__ wg,
                                                  const float *__restrict__ bg,
                                                  float *__restrict__ partial,
                                                  float *__restrict__ loss_partial) {
    typedef typename Prec<F>::W WT;
    __shared__ WT W[kWpad];
    __shared__ float b[kBpad];
    __shared__ float G[kGpad];
    __shared__ WT Tz[16 * 64], Th[16 * 64];
    load_weights_lds(wg, bg, W, b);
    for (int i = threadIdx.x; i < kGpad; i += blockDim.x) G[i] = 0.f;
    __syncthreads();
    const int l = threadIdx.x, g = l >> 4;
    const int64_t ntiles = (B + 15) / 16;
    float lsum = 0.f;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        Fwd<F> f;
        mlp_tile_forward<F>(W, b, X, B, 16 * t, l, f);
        const int64_t s = 16 * t + (l & 15);
        const bool valid = s < B;
        // dZ4 = (y - t) * scale on rows 0..2
        f32x4 dz4 = {0.f, 0.f, 0.f, 0.f};
        if (g == 0 && valid)
            for (int r = 0; r < 3; r++) {
                float d = f.y[r] - T[3 * s + r];
                lsum += 0.5f * d * d * scale;
                dz4[r] = d * scale;
            }
        // layer 4: dW4 (16 x 64) += dZ4^T H3
        typename Prec<F>::Op dz4b = to_op<F>(dz4);
        for (int ob = 0; ob < 4; ob++) {
            f32x4 h = f.z3[ob];
            for (int r = 0; r < 4; r++) h[r] = valid ? silu(h[r]) : 0.f;
            store_tile<F>(Th, 64, ob, h, l);
        }
        store_tile<F>(Tz, 16, 0, dz4, l);
        __syncthreads();
        acc_dw<F>(Tz, 16, Th, 64, G + kW4p, l);
        acc_db(dz4, G, kWpad + kB4p, 0, l);
        __syncthreads();
        // dH3 = W4^T dZ4 ; dZ3 = dH3 * silu'(z3)
        f32x4 dz[4];
        for (int ob = 0; ob < 4; ob++) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma16<F>(load_at<F>(W + kW4p, 64, 16 * ob, 0, l), dz4b, acc);
            for (int r = 0; r < 4; r++) acc[r] *= dsilu(f.z3[ob][r]);
            dz[ob] = acc;
        }
        // layers 3 and 2: dW += dZ^T H(prev); dZ(prev) = (W^T dZ) * silu'(z(prev))
        hidden_back<F>(W, G, kW3, kB3, f.z2, dz, Tz, Th, valid, l);
        hidden_back<F>(W, G, kW2, kB2, f.z1, dz, Tz, Th, valid, l);
        // layer 1: dW1p (64 x 16) += dZ1^T Xp
        for (int r = 0; r < 4; r++) Th[(l & 15) * 16 + 4 * g + r] = (WT)f.x[r];
        for (int ob = 0; ob < 4; ob++) store_tile<F>(Tz, 64, ob, dz[ob], l);
        __syncthreads();
        acc_dw<F>(Tz, 64, Th, 16, G + kW1p, l);
        for (int ob = 0; ob < 4; ob++) acc_db(dz[ob], G, kWpad + kB1, ob, l);
        __syncthreads();
    }
    float* out = partial + (size_t)blockIdx.x * kGpad;
    for (int i = threadIdx.x; i < kGpad; i += blockDim.x) out[i] = G[i];
    for (int m = 1; m < 64; m <<= 1) lsum += __shfl_xor(lsum, m, 64);
    if (threadIdx.x == 0) loss_partial[blockIdx.x] = lsum;
}

// Sum of the workgroup partials in a fixed order: block j < kGpad / 64 owns
// 64 consecutive entries of the padded gradient image; its 4 thread groups
// sum 4 contiguous quarters of the partials (coalesced rows) and the quarter
// sums are added in order.  The extra last block sums the loss partials
// (fixed per-thread strides, then a fixed tree).
constexpr int kRedCols = 64;
constexpr int kRedBlocks = (kGpad + kRedCols - 1) / kRedCols;

__global__ __launch_bounds__(256) void k_mlp_reduce_pad(int nb, const float *__restrict__ partial,
                                                       const float *__restrict__ loss_partial,
                                                       float *__restrict__ gpad,
                                                       float *__restrict__ loss) {
    __shared__ float sh[256];
    const int t = threadIdx.x;
    if (blockIdx.x == kRedBlocks) {
        float s = 0.f;
        for (int k = t; k < nb; k += 256) s += loss_partial[k];
        sh[t] = s;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) sh[t] += sh[t + o];
            __syncthreads();
        }
        if (t == 0) *loss = sh[0];
        return;
    }
    const int c = t % kRedCols, g = t / kRedCols;
    const int i = blockIdx.x * kRedCols + c;
    const int q = (nb + 3) / 4, k0 = g * q, k1 = k0 + q < nb ? k0 + q : nb;
    float s = 0.f;
    if (i < kGpad)
        for (int k = k0; k < k1; k++) s += partial[(size_t)k * kGpad + i];
    sh[t] = s;
    __syncthreads();
    if (g == 0 && i < kGpad) gpad[i] = (sh[c] + sh[64 + c]) + (sh[128 + c] + sh[192 + c]);
}

// fold the padded gradient image back to the master layout
__global__ void k_mlp_fold(const float *__restrict__ gp, float *__restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNP) return;
    float v;
    if (i < 512) {                               // W1[o][c]: both copies of column c
        int o = i / 8, c = i % 8;
        v = gp[kW1p + o * 16 + c] + gp[kW1p + o * 16 + 8 + c];
    } else if (i < 576) v = gp[kWpad + kB1 + (i - 512)];
    else if (i < 4672) v = gp[kW2 + (i - 576)];
    else if (i < 4736) v = gp[kWpad + kB2 + (i - 4672)];
    else if (i < 8832) v = gp[kW3 + (i - 4736)];
    else if (i < 8896) v = gp[kWpad + kB3 + (i - 8832)];
    else if (i < 9088) v = gp[kW4p + (i - 8896)];    // rows 0..2 of W4p
    else v = gp[kWpad + kB4p + (i - 9088)];
    grad[i] = v;
}

// master FP32 -> padded BF16 weights (and the same image in FP32, for the
// FP32 debug mode) + FP32 biases
__global__ void k_mlp_pack(const float *__restrict__ P, unsigned short *__restrict__ wg,
                           float *__restrict__ wf, float *__restrict__ bg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kWpad) {
        float v = 0.f;
        if (i < kW2) { int o = i / 16, c = i % 16; v = P[o * 8 + (c & 7)]; }
        else if (i < kW3) v = P[576 + (i - kW2)];
        else if (i < kW4p) v = P[4736 + (i - kW3)];
        else { int o = (i - kW4p) / 64, c = (i - kW4p) % 64; v = o < 3 ? P[8896 + o * 64 + c] : 0.f; }
        wg[i] = f2bf(v);
        wf[i] = v;
    }
    if (i < kBpad) {
        float v;
        if (i < 64) v = P[512 + i];
        else if (i < 128) v = P[4672 + i - 64];
        else if (i < 192) v = P[8832 + i - 128];
        else v = (i - 192) < 3 ? P[9088 + i - 192] : 0.f;
        bg[i] = v;
    }
}

__global__ void k_adam(int n, float *__restrict__ P, const float *__restrict__ G,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float g = G[i];
    float mi = b1 * m[i] + (1.f - b1) * g;
    float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace bs

// ------------------------------------------------------------------ C ABI
using namespace bs;

struct bs_mlp_s {
    hipStream_t stream = nullptr;
    float *P = nullptr, *m = nullptr, *v = nullptr, *G = nullptr;
    unsigned short *wg = nullptr;
    float *wf = nullptr;     // FP32 image of the padded weights (debug mode)
    float *bg = nullptr;
    int fp32 = 0;            // 1: FP32 weights and activations (debug mode)
    float *partial = nullptr, *loss_partial = nullptr, *loss = nullptr, *gpad = nullptr;
    int nb = 512;
    int64_t step = 0;
    std::string err;
};

namespace bs {
hipStream_t mlp_stream(bs_mlp_t M) { return M->stream; }

void mlp_forward_device(bs_mlp_t M, const int *Bdev, int64_t Bmax, const float *X, float *Y,
                        hipStream_t stream) {
    int64_t tiles = (Bmax + 15) / 16;
    int blocks = (int)std::min<int64_t>(std::max<int64_t>((tiles + 3) / 4, 1), 2048);
    if (M->fp32)
        hipLaunchKernelGGL(k_mlp_infer<true>, dim3(blocks), dim3(256), 0, stream, Bmax, Bdev, X,
                           (const float *)M->wf, M->bg, Y);
    else
        hipLaunchKernelGGL(k_mlp_infer<false>, dim3(blocks), dim3(256), 0, stream, Bmax, Bdev, X,
                           (const unsigned short *)M->wg, M->bg, Y);
}
}  // namespace bs

extern "C" {

int bs_mlp_nparams(void) { return kNP; }

int bs_mlp_create(const float *params_host, void *hip_stream, bs_mlp_t *out) {
    if (!out || !params_host) return BS_EINVAL;
    bs_mlp_t M = new bs_mlp_s();
    M->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    auto al = [&](void **p, size_t bytes) { if (e == hipSuccess) e = hipMalloc(p, bytes); };
    al((void **)&M->P, kNP * 4); al((void **)&M->m, kNP * 4); al((void **)&M->v, kNP * 4);
    al((void **)&M->G, kNP * 4); al((void **)&M->wg, kWpad * 2); al((void **)&M->bg, kBpad * 4);
    al((void **)&M->wf, kWpad * 4);
    al((void **)&M->partial, (size_t)M->nb * kGpad * 4);
    al((void **)&M->loss_partial, M->nb * 4); al((void **)&M->loss, 4);
    al((void **)&M->gpad, kGpad * 4);
    if (e != hipSuccess) { bs_mlp_destroy(M); return BS_ENOMEM; }
    (void)hipMemcpy(M->P, params_host, kNP * 4, hipMemcpyHostToDevice);
    (void)hipMemset(M->m, 0, kNP * 4);
    (void)hipMemset(M->v, 0, kNP * 4);
    hipLaunchKernelGGL(k_mlp_pack, dim3(ceil_div(kWpad, 256)), dim3(256), 0, M->stream, M->P,
                       M->wg, M->wf, M->bg);
    *out = M;
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

int bs_mlp_forward(bs_mlp_t M, int64_t B, const float *X, float *Y) {
    if (!M || B < 0 || (B > 0 && (!X || !Y))) return BS_EINVAL;
    if (B == 0) return BS_OK;
    int64_t tiles = (B + 15) / 16;
    int blocks = (int)std::min<int64_t>((tiles + 3) / 4, 4096);
    if (M->fp32)
        hipLaunchKernelGGL(k_mlp_infer<true>, dim3(blocks), dim3(256), 0, M->stream, B,
                           (const int *)nullptr, X, (const float *)M->wf, M->bg, Y);
    else
        hipLaunchKernelGGL(k_mlp_infer<false>, dim3(blocks), dim3(256), 0, M->stream, B,
                           (const int *)nullptr, X, (const unsigned short *)M->wg, M->bg, Y);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

static int mlp_grad(bs_mlp_t M, int64_t B, const float *X, const float *T) {
    int64_t tiles = (B + 15) / 16;
    int blocks = (int)std::min<int64_t>(tiles, M->nb);
    if (M->fp32)
        hipLaunchKernelGGL(k_mlp_train<true>, dim3(blocks), dim3(64), 0, M->stream, B, X, T,
                           1.0f / (float)B, (const float *)M->wf, M->bg, M->partial,
                           M->loss_partial);
    else
        hipLaunchKernelGGL(k_mlp_train<false>, dim3(blocks), dim3(64), 0, M->stream, B, X, T,
                           1.0f / (float)B, (const unsigned short *)M->wg, M->bg, M->partial,
                           M->loss_partial);
    hipLaunchKernelGGL(k_mlp_reduce_pad, dim3(kRedBlocks + 1), dim3(256), 0, M->stream, blocks,
                       M->partial, M->loss_partial, M->gpad, M->loss);
    hipLaunchKernelGGL(k_mlp_fold, dim3(ceil_div(kNP, 256)), dim3(256), 0, M->stream, M->gpad,
                       M->G);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

int bs_mlp_loss_grad(bs_mlp_t M, int64_t B, const float *X, const float *T, float *loss_dev,
                     float *grad_dev) {
    if (!M || B <= 0 || !X || !T) return BS_EINVAL;
    int rc = mlp_grad(M, B, X, T);
    if (rc) return rc;
    if (loss_dev) (void)hipMemcpyAsync(loss_dev, M->loss, 4, hipMemcpyDeviceToDevice, M->stream);
    if (grad_dev) (void)hipMemcpyAsync(grad_dev, M->G, kNP * 4, hipMemcpyDeviceToDevice, M->stream);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

int bs_mlp_adam_step(bs_mlp_t M, int64_t B, const float *X, const float *T, float lr,
                     float beta1, float beta2, float eps, float *loss_dev) {
    if (!M || B <= 0 || !X || !T) return BS_EINVAL;
    int rc = mlp_grad(M, B, X, T);
    if (rc) return rc;
    M->step++;
    float c1 = 1.f - powf(beta1, (float)M->step), c2 = 1.f - powf(beta2, (float)M->step);
    hipLaunchKernelGGL(k_adam, dim3(ceil_div(kNP, 256)), dim3(256), 0, M->stream, kNP, M->P, M->G,
                       M->m, M->v, lr, beta1, beta2, eps, c1, c2);
    hipLaunchKernelGGL(k_mlp_pack, dim3(ceil_div(kWpad, 256)), dim3(256), 0, M->stream, M->P,
                       M->wg, M->wf, M->bg);
    if (loss_dev) (void)hipMemcpyAsync(loss_dev, M->loss, 4, hipMemcpyDeviceToDevice, M->stream);
    return hipGetLastError() == hipSuccess ? BS_OK : BS_EDEVICE;
}

int bs_mlp_set_fp32(bs_mlp_t M, int enable) {
    if (!M) return BS_EINVAL;
    M->fp32 = enable ? 1 : 0;
    return BS_OK;
}

int bs_mlp_get_params(bs_mlp_t M, float *params_host) {
    if (!M || !params_host) return BS_EINVAL;
    (void)hipStreamSynchronize(M->stream);
    return hipMemcpy(params_host, M->P, kNP * 4, hipMemcpyDeviceToHost) == hipSuccess ? BS_OK
                                                                                   : BS_EDEVICE;
}

int bs_mlp_destroy(bs_mlp_t M) {
    if (!M) return BS_OK;
    (void)hipStreamSynchronize(M->stream);
    void *all[] = {M->P, M->m, M->v, M->G, M->wg, M->wf, M->bg, M->partial, M->loss_partial,
                   M->loss, M->gpad};
    for (void *p : all)
        if (p) (void)hipFree(p);
    delete M;
    return BS_OK;
}

}  // extern "C"
