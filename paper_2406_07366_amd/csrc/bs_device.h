// Device helpers shared by the binning, NUFFT and pair kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace bs {

// Position folded into [0, L).  Anything that does not land there (NaN,
// infinities, magnitudes where the fold loses all digits) maps to 0, so that
// every index derived from the result stays inside its array; such input is
// reported through the plan's status word by the chord-length kernel.
__device__ __forceinline__ double wrap_box(double v, double L) {
    double r = v - L * floor(v / L);
    if (r >= L) r -= L;
    return (r >= 0.0 && r < L) ? r : 0.0;
}

// Stencil base per axis: i0 = floor(u - w/2) + 1 with u = x/h, x wrapped
// to [0, L); the support is i0 .. i0 + w - 1 (mod n).
__device__ __forceinline__ int stencil_base(double xw, double inv_h, int w, int n, double *frac) {
    double u = xw * inv_h;
    double i0 = floor(u - 0.5 * w) + 1.0;
    *frac = u - i0;
    int b = (int)i0 % n;
    return b < 0 ? b + n : b;
}

// spread-tile key of a quadrature point and pair-cell key of a position
__device__ __forceinline__ int tile_key(const double *p, double L, double inv_h, int w, int n,
                                        int T, int NT) {
    double f;
    const int bx = stencil_base(wrap_box(p[0], L), inv_h, w, n, &f);
    const int by = stencil_base(wrap_box(p[1], L), inv_h, w, n, &f);
    const int bz = stencil_base(wrap_box(p[2], L), inv_h, w, n, &f);
    return ((bz / T) * NT + by / T) * NT + bx / T;
}
__device__ __forceinline__ int cell_key(const double *p, double L, int nc) {
    int c[3];
    for (int q = 0; q < 3; q++) {
        const int v = (int)(wrap_box(p[q], L) / L * nc);
        c[q] = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
    }
    return (c[2] * nc + c[1]) * nc + c[0];
}

// Backward Kaiser-Bessel kernel, normalised to 1 at the centre:
//   phi(z) = sinh(zeta sqrt(1-z^2)) / (sinh(zeta) sqrt(1-z^2)),  |z| <= 1
// (eq:kaiser_bessel_bw up to the constant pi/sinh(zeta), which the
// deconvolution table carries).  Written as
//   exp(zeta (s-1)) * (1 - exp(-2 zeta s)) / ((1 - exp(-2 zeta)) s)
// with 1 - exp(-y) = -expm1(-y) to keep digits as s -> 0.
__device__ __forceinline__ double kb_phi(double z, double zeta, double inv_den) {
    double s2 = 1.0 - z * z;
    if (s2 <= 0.0) return 2.0 * zeta * exp(-zeta) * inv_den;
    double s = sqrt(s2);
    return exp(zeta * (s - 1.0)) * (-expm1(-2.0 * zeta * s)) / s * inv_den;
}


__device__ __forceinline__ int next_node_d(const int *off, const int *fil, int j) {
    int f = fil[j];
    return (j + 1 < off[f + 1]) ? j + 1 : off[f];
}
__device__ __forceinline__ int prev_node_d(const int *off, const int *fil, int j) {
    int f = fil[j];
    return (j > off[f]) ? j - 1 : off[f + 1] - 1;
}

// Workgroups are dispatched round-robin over the 8 XCDs, so blocks b, b+8,
// b+16, ... run on one XCD.  With the grid launched as 8 * per blocks, this
// maps them to the consecutive logical indices [xcd * per, (xcd + 1) * per),
// so neighbouring logical blocks share an L2.  Indices >= the real count
// must exit (uniformly over the block).
// LDS written by some lanes of a wavefront and read by others of the same
// wavefront: wait for the stores and keep the compiler from moving memory
// operations across.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int xcd_block(int per) {
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// Groups of the active lanes of a wavefront with equal (tag, tag2): each lane
// learns its group's lowest lane (itself when inactive) and its rank in the
// group in lane order; the lowest lane also learns the group size.  No
// memory access: the callers then issue one atomic per group, all groups at
// once, so a wavefront waits for one atomic round trip whatever the number
// of distinct keys.  Call from converged control flow (every lane).
struct WaveGroup {
    int leader, rank, size;
};
__device__ __forceinline__ WaveGroup wave_group(int tag, int tag2, bool active) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long todo = __ballot(active);
    WaveGroup g{lane, 0, 0};
    while (todo) {
        const int l = __ffsll((long long)todo) - 1;
        const int tl = __shfl(tag, l), tl2 = __shfl(tag2, l);
        const unsigned long long grp = __ballot(active && tag == tl && tag2 == tl2) & todo;
        if ((grp >> lane) & 1ull) {
            g.leader = l;
            g.rank = __popcll(grp & below);
        }
        if (lane == l) g.size = __popcll(grp);
        todo &= ~grp;
    }
    return g;
}

// counter[key] += 1 for every active lane, with one atomic per distinct key
// in the wavefront (the group's lowest lane adds the group size).  With RET,
// returns the counter's value before the lane's own increment (the group's
// old value plus the lane's rank in the group, in lane order); else 0.  Call
// from converged control flow, with active false for lanes that have no item.
template <bool RET>
__device__ __forceinline__ int wave_add(int *counter, int key, bool active) {
    const WaveGroup g = wave_group(key, 0, active);
    const int lane = threadIdx.x & 63;
    int old = 0;
    if (active && lane == g.leader) {
        if (RET) old = atomicAdd(counter + key, g.size);
        else atomicAdd(counter + key, g.size);
    }
    if (!RET) return 0;
    return __shfl(old, g.leader) + g.rank;
}

// Orders the distinct entries perm[s .. s+n) ascending: every entry's rank is
// the number of smaller entries in the bin, and it is written to its rank slot.
// Called by a whole workgroup for one bin.  Bins of up to CAP entries are
// ranked from the LDS array v and written back in place; larger bins are
// ranked from global memory into scratch (same indexing) and copied back.
template <int CAP>
__device__ void rank_sort_bin(int *perm, int *scratch, int s, int n, int *v) {
    if (n <= 1) return;
    if (n <= CAP) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = perm[s + i];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int xv = v[i], r = 0;
            for (int j = 0; j < n; j++) r += (v[j] < xv);
            perm[s + r] = xv;
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int xv = perm[s + i], r = 0;
        for (int j = 0; j < n; j++) r += (perm[s + j] < xv);
        scratch[s + r] = xv;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[s + i] = scratch[s + i];
}

}  // namespace bs

namespace bs {

// ------------------------------------------------------------ spline segments
// Segment j of a filament in the local coordinate u in [0, 1]
// (tau = tau_j + u h_j): s(u) = sum_k c_k u^k, built from the node values s,
// slopes D = ds/dtau and (quintic only) second derivatives S = d2s/dtau2 at
// both ends.  ORDER 4: the cubic Hermite segment of the C2 spline; ORDER 6:
// the quintic Hermite segment of the C4 spline (both are the periodic
// interpolating splines of App. B on the chord-length knots).
template <int ORDER>
struct SegPoly {
    double c[ORDER][3];

    // s0 = x[j], s1 = xe[je] (the end node in the segment's own frame);
    // D, S at nodes j and jn
    __device__ __forceinline__ void load(const double *__restrict__ x,
                                         const double *__restrict__ xe, int je,
                                         const double *__restrict__ D,
                                         const double *__restrict__ S, int j, int jn, double h) {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const double s0 = x[3 * j + q], s1 = xe[3 * je + q];
            const double d0 = h * D[3 * j + q], d1 = h * D[3 * jn + q];
            c[0][q] = s0;
            c[1][q] = d0;
            if constexpr (ORDER == 4) {
                c[2][q] = 3.0 * (s1 - s0) - 2.0 * d0 - d1;
                c[3][q] = 2.0 * (s0 - s1) + d0 + d1;
            } else {
                // matches s1, h D1, h^2 S1 at u = 1: with A, B, C the
                // misfits of the value, slope and curvature of the
                // quadratic part there
                const double q0 = h * h * S[3 * j + q], q1 = h * h * S[3 * jn + q];
                const double A = s1 - s0 - d0 - 0.5 * q0, B = d1 - d0 - q0, C = q1 - q0;
                c[2][q] = 0.5 * q0;
                c[3][q] = 10.0 * A - 4.0 * B + 0.5 * C;
                c[4][q] = -15.0 * A + 7.0 * B - C;
                c[5][q] = 6.0 * A - 3.0 * B + 0.5 * C;
            }
        }
    }
    // s(u)
    __device__ __forceinline__ void pos(double u, double *p) const {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            double v = c[ORDER - 1][q];
#pragma unroll
            for (int k = ORDER - 2; k >= 0; k--) v = v * u + c[k][q];
            p[q] = v;
        }
    }
    // ds/du (divide by h for ds/dtau)
    __device__ __forceinline__ void der(double u, double *d) const {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            double v = (ORDER - 1) * c[ORDER - 1][q];
#pragma unroll
            for (int k = ORDER - 2; k >= 1; k--) v = v * u + k * c[k][q];
            d[q] = v;
        }
    }
    // d2s/du2 (divide by h^2 for d2s/dtau2)
    __device__ __forceinline__ void der2(double u, double *d) const {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            double v = (ORDER - 1) * (ORDER - 2) * c[ORDER - 1][q];
#pragma unroll
            for (int k = ORDER - 2; k >= 2; k--) v = v * u + k * (k - 1) * c[k][q];
            d[q] = v;
        }
    }
};

}  // namespace bs
