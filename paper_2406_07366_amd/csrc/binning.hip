// Binning of quadrature points and nodes (counting sort), and the sorted
// structure-of-arrays copies that the spread, interpolation and pair kernels
// read.
//
//   spread bins : tile of T^3 grid cells containing a point's stencil base
//                 (lowest grid index of its w-point support per axis);
//   pair cells  : ncell^3 cells of edge L/ncell >= r_c (the cell-list idea of
//                 Sec. 5.3, with cells no smaller than r_c so that the 27
//                 surrounding cells hold every pair within r_c);
//   node order  : nodes sorted by pair cell, so neighbouring threads share
//                 cells in the pair and interpolation kernels.
//
// Within a bin, entries are ordered by original index so that every sum the
// later kernels form has a fixed order (bitwise reproducible results).
#include "bs_internal.h"
#include "bs_device.h"

namespace bs {

// ------------------------------------------------------------ scan (int32)
constexpr int kScanBlock = 256, kScanItems = 8, kScanTile = kScanBlock * kScanItems;

__device__ int block_exclusive_scan(int v, int *sh, int *total) {
    // Hillis-Steele scan over the block in LDS
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < blockDim.x; o <<= 1) {
        int add = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int incl = sh[t];
    *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_reduce(const int *__restrict__ in, int n, int *__restrict__ sums) {
    __shared__ int sh[kScanBlock];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += in[base + k];
    int tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int *__restrict__ sums, int nb, int *__restrict__ total_out) {
    __shared__ int sh[kScanBlock];
    // nb <= kScanTile
    int base = threadIdx.x * kScanItems;
    int v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < nb) ? sums[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, sh, &tot);
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < nb) sums[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) *total_out = tot;
}

__global__ void k_scan_apply(const int *__restrict__ in, int n, const int *__restrict__ sums,
                             int *__restrict__ out) {
    __shared__ int sh[kScanBlock];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, sh, &tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

// out[0..n-1] = exclusive scan of in, out[n] = total.  in and out may not
// alias.  Requires n <= kScanTile^2 (4.2 M bins).
void exclusive_scan(bs_plan_t p, const int *in, int *out, int n) {
    int nb = ceil_div(n, kScanTile);
    int *sums = (int *)p->red_tmp.p;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, p->stream, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, p->stream, sums, nb, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanBlock), 0, p->stream, in, n, sums, out);
}

// ---------------------------------------------------------------- keys
__global__ void k_keys_spread(int M, const double *__restrict__ pos, double L, double inv_h,
                              int w, int n, int T, int NT, int *__restrict__ key,
                              int *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double f;
    int bx = stencil_base(wrap_box(pos[3 * i], L), inv_h, w, n, &f);
    int by = stencil_base(wrap_box(pos[3 * i + 1], L), inv_h, w, n, &f);
    int bz = stencil_base(wrap_box(pos[3 * i + 2], L), inv_h, w, n, &f);
    int k = ((bz / T) * NT + by / T) * NT + bx / T;
    key[i] = k;
    atomicAdd(&cnt[k], 1);
}

__global__ void k_keys_cell(int M, const double *__restrict__ pos, double L, int nc,
                            int *__restrict__ key, int *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int c[3];
    for (int q = 0; q < 3; q++) {
        int v = (int)(wrap_box(pos[3 * i + q], L) / L * nc);
        c[q] = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
    }
    int k = (c[2] * nc + c[1]) * nc + c[0];
    key[i] = k;
    atomicAdd(&cnt[k], 1);
}

__global__ void k_scatter(int M, const int *__restrict__ key, const int *__restrict__ start,
                          int *__restrict__ fill, int *__restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int k = key[i];
    perm[start[k] + atomicAdd(&fill[k], 1)] = i;
}

// Order each bin by original index: one wavefront per bin computes every
// entry's rank (number of smaller indices in the bin) and writes it to its
// rank slot.  Bins of up to kSortLds entries are ranked in LDS and written
// back in place; larger bins are ranked from global memory into `scratch`
// (the key array, free once the scatter is done) and copied back.
constexpr int kSortLds = 2048;

__global__ __launch_bounds__(64) void k_sort_bins(int nbins, const int *__restrict__ start,
                                                  int *__restrict__ perm,
                                                  int *__restrict__ scratch) {
    __shared__ int v[kSortLds];
    int b = blockIdx.x;
    if (b >= nbins) return;
    int s = start[b], n = start[b + 1] - s;
    if (n <= 1) return;
    if (n <= kSortLds) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = perm[s + i];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            int x = v[i], r = 0;
            for (int j = 0; j < n; j++) r += (v[j] < x);
            perm[s + r] = x;
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int x = perm[s + i], r = 0;
        for (int j = 0; j < n; j++) r += (perm[s + j] < x);
        scratch[s + r] = x;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[s + i] = scratch[s + i];
}

__global__ void k_fill_int(int *p, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// -------------------------------------------------- sorted copies for spread
template <typename R>
__global__ void k_gather_spread(int M, int w, const int *__restrict__ perm,
                                const double *__restrict__ pos, const double *__restrict__ chg,
                                double L, double inv_h, int n, double zeta, double inv_den,
                                int4 *__restrict__ base, R *__restrict__ ker,
                                R *__restrict__ q) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    int o = perm[p];
    int b[3];
    double half = 0.5 * w;
    for (int d = 0; d < 3; d++) {
        double f;
        b[d] = stencil_base(wrap_box(pos[3 * o + d], L), inv_h, w, n, &f);
        for (int k = 0; k < w; k++)
            ker[((size_t)p * 3 + d) * w + k] = (R)kb_phi((k - f) / half, zeta, inv_den);
    }
    base[p] = make_int4(b[0], b[1], b[2], 0);
    q[4 * (size_t)p + 0] = (R)chg[3 * o + 0];
    q[4 * (size_t)p + 1] = (R)chg[3 * o + 1];
    q[4 * (size_t)p + 2] = (R)chg[3 * o + 2];
    q[4 * (size_t)p + 3] = (R)0;
}

// ---------------------------------------------------- sorted copies for pairs
template <typename R>
__global__ void k_gather_pairs(int M, int Q, const int *__restrict__ perm,
                               const double *__restrict__ pos, const double *__restrict__ chg,
                               double L, double4 *__restrict__ spos, R *__restrict__ schg,
                               int *__restrict__ sseg) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    int o = perm[p];
    spos[p] = make_double4(wrap_box(pos[3 * o], L), wrap_box(pos[3 * o + 1], L),
                           wrap_box(pos[3 * o + 2], L), 0.0);
    schg[4 * (size_t)p + 0] = (R)chg[3 * o + 0];
    schg[4 * (size_t)p + 1] = (R)chg[3 * o + 1];
    schg[4 * (size_t)p + 2] = (R)chg[3 * o + 2];
    schg[4 * (size_t)p + 3] = (R)0;
    sseg[p] = o / Q;
}

// ---------------------------------------------------------------- driver
static void zero_bins(bs_plan_t p, int nbins, int *cnt, int *fill) {
    int bs = 256;
    hipLaunchKernelGGL(k_fill_int, dim3(ceil_div(nbins, bs)), dim3(bs), 0, p->stream, cnt, nbins, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(ceil_div(nbins, bs)), dim3(bs), 0, p->stream, fill, nbins, 0);
}

void build_bins(bs_plan_t p) {
    const int bs = 256;
    const int M = (int)p->Nq, N = (int)p->N;
    const double L = p->prm.L, inv_h = p->n / L;
    const int w = p->prm.w, n = p->n;
    // --- spread tiles
    int ntiles = p->NT * p->NT * p->NT;
    int *key = (int *)p->sp_key.p, *cnt = (int *)p->sp_cnt.p, *start = (int *)p->sp_start.p,
        *fill = (int *)p->sp_fill.p, *perm = (int *)p->sp_perm.p;
    zero_bins(p, ntiles, cnt, fill);
    hipLaunchKernelGGL(k_keys_spread, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream, M,
                       (const double *)p->d_qpos.p, L, inv_h, w, n, p->T, p->NT, key, cnt);
    exclusive_scan(p, cnt, start, ntiles);
    hipLaunchKernelGGL(k_scatter, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream, M, key, start,
                       fill, perm);
    hipLaunchKernelGGL(k_sort_bins, dim3(ntiles), dim3(64), 0, p->stream, ntiles, start, perm,
                       key);
    const double zeta = p->prm.zeta, inv_den = 1.0 / (-expm1(-2.0 * zeta));
    if (p->fp32)
        hipLaunchKernelGGL(k_gather_spread<float>, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream,
                           M, w, perm, (const double *)p->d_qpos.p, (const double *)p->d_qchg.p,
                           L, inv_h, n, zeta, inv_den, (int4 *)p->sp_base.p,
                           (float *)p->sp_ker.p, (float *)p->sp_q.p);
    else
        hipLaunchKernelGGL(k_gather_spread<double>, dim3(ceil_div(M, bs)), dim3(bs), 0,
                           p->stream, M, w, perm, (const double *)p->d_qpos.p,
                           (const double *)p->d_qchg.p, L, inv_h, n, zeta, inv_den,
                           (int4 *)p->sp_base.p, (double *)p->sp_ker.p, (double *)p->sp_q.p);

    // --- pair cells for quadrature points
    int nc3 = p->nc * p->nc * p->nc;
    key = (int *)p->pq_key.p; cnt = (int *)p->pq_cnt.p; start = (int *)p->pq_start.p;
    fill = (int *)p->pq_fill.p; perm = (int *)p->pq_perm.p;
    zero_bins(p, nc3, cnt, fill);
    hipLaunchKernelGGL(k_keys_cell, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream, M,
                       (const double *)p->d_qpos.p, L, p->nc, key, cnt);
    exclusive_scan(p, cnt, start, nc3);
    hipLaunchKernelGGL(k_scatter, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream, M, key, start,
                       fill, perm);
    hipLaunchKernelGGL(k_sort_bins, dim3(nc3), dim3(64), 0, p->stream, nc3, start, perm, key);
    if (p->fp32)
        hipLaunchKernelGGL(k_gather_pairs<float>, dim3(ceil_div(M, bs)), dim3(bs), 0, p->stream,
                           M, p->Q, perm, (const double *)p->d_qpos.p,
                           (const double *)p->d_qchg.p, L, (double4 *)p->pq_pos.p,
                           (float *)p->pq_chg.p, (int *)p->pq_seg.p);
    else
        hipLaunchKernelGGL(k_gather_pairs<double>, dim3(ceil_div(M, bs)), dim3(bs), 0,
                           p->stream, M, p->Q, perm, (const double *)p->d_qpos.p,
                           (const double *)p->d_qchg.p, L, (double4 *)p->pq_pos.p,
                           (double *)p->pq_chg.p, (int *)p->pq_seg.p);

    // --- nodes by pair cell
    key = (int *)p->nd_key.p; cnt = (int *)p->nd_cnt.p; start = (int *)p->nd_start.p;
    fill = (int *)p->nd_fill.p; perm = (int *)p->nd_perm.p;
    zero_bins(p, nc3, cnt, fill);
    hipLaunchKernelGGL(k_keys_cell, dim3(ceil_div(N, bs)), dim3(bs), 0, p->stream, N,
                       (const double *)p->d_x.p, L, p->nc, key, cnt);
    exclusive_scan(p, cnt, start, nc3);
    hipLaunchKernelGGL(k_scatter, dim3(ceil_div(N, bs)), dim3(bs), 0, p->stream, N, key, start,
                       fill, perm);
    hipLaunchKernelGGL(k_sort_bins, dim3(nc3), dim3(64), 0, p->stream, nc3, start, perm, key);
}

}  // namespace bs
