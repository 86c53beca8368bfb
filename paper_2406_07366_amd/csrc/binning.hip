// Binning of quadrature points and nodes (counting sort), and the sorted
// structure-of-arrays copies that the spread, interpolation and pair kernels
// read.
//
//   spread bins : tile of T^3 grid cells containing a point's stencil base
//                 (lowest grid index of its w-point support per axis);
//   pair cells  : ncell^3 cells of edge L/ncell >= 2 r_c / 3 (the cell-list
//                 idea of Sec. 5.3), so that the 4 x 4 x 4 cells from the
//                 cell of x - r_c on hold every point within r_c of x;
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
// alias.  Requires n <= kScanTile^2 (4.2 M bins); sums: kScanTile ints of
// scratch, private to the stream.
void exclusive_scan(bs_plan_t p, const int *in, int *out, int n, int *sums) {
    int nb = ceil_div(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, p->stream, in, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, p->stream, sums, nb, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanBlock), 0, p->stream, in, n, sums, out);
}

// Bins are ordered by original index: one wavefront per bin ranks its
// entries (rank_sort_bin); a bin too large for LDS ranks into the key array,
// which is free once the scatter is done.
constexpr int kSortLds = 2048;

// ------------------------------------------------------- fused bin passes
// The three sorts (quadrature points by spread tile, quadrature points by pair
// cell, nodes by pair cell) run side by side: each pass below is one launch
// covering all three.
struct SortSet {
    int *key[3], *cnt[3], *start[3], *fill[3], *perm[3];
    int nbins[3], nitems[3];
};


// one workgroup per array: exclusive scan of cnt into start (start[n] =
// total).  Wavefront w owns the contiguous segment [w seg, (w + 1) seg) and
// reads it 64 entries at a time (coalesced): a first pass sums it, the
// segment offsets are formed from the 16 sums in LDS, and a second pass
// scans each 64-entry chunk by shuffles while writing.
__global__ __launch_bounds__(1024) void k_scan_small(SortSet S) {
    __shared__ int wsum[16];
    const int a = blockIdx.x;
    const int n = S.nbins[a];
    const int *in = S.cnt[a];
    int *out = S.start[a];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int seg = ((n + nw - 1) / nw + 63) / 64 * 64;
    const int b0 = wave * seg, b1 = b0 + seg < n ? b0 + seg : n;
    int sum = 0;
    for (int i = b0 + lane; i < b1; i += 64) sum += in[i];
    for (int m = 32; m > 0; m >>= 1) sum += __shfl_xor(sum, m);
    if (lane == 0) wsum[wave] = sum;
    __syncthreads();
    int carry = 0;
    for (int w = 0; w < wave; w++) carry += wsum[w];
    for (int c0 = b0; c0 < b1; c0 += 64) {
        const int i = c0 + lane;
        const int v = i < b1 ? in[i] : 0;
        int incl = v;
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d);
            if (lane >= d) incl += u;
        }
        if (i < b1) out[i] = carry + incl - v;
        carry += __shfl(incl, 63);
    }
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < nw; w++) tot += wsum[w];
        out[n] = tot;
    }
}

__global__ void k_scatter_all(SortSet S) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int a = 0;
    if (i >= S.nitems[0]) { i -= S.nitems[0]; a = 1; }
    if (a == 1 && i >= S.nitems[1]) { i -= S.nitems[1]; a = 2; }
    const bool valid = !(a == 2 && i >= S.nitems[2]);
    const int k = valid ? S.key[a][i] : 0;
    // one atomic per (set, bin) group of the wavefront, all issued together
    const WaveGroup g = wave_group(k, a, valid);
    int old = 0;
    if (valid && (int)(threadIdx.x & 63) == g.leader) old = atomicAdd(S.fill[a] + k, g.size);
    const int slot = __shfl(old, g.leader) + g.rank;
    if (valid) S.perm[a][S.start[a][k] + slot] = i;
}

__global__ __launch_bounds__(64) void k_sort_all(SortSet S) {
    int b = blockIdx.x, a = 0;
    if (b >= S.nbins[0]) { b -= S.nbins[0]; a = 1; }
    if (a == 1 && b >= S.nbins[1]) { b -= S.nbins[1]; a = 2; }
    if (a == 2 && b >= S.nbins[2]) return;
    __shared__ int v[kSortLds];
    int s = S.start[a][b], n = S.start[a][b + 1] - s;
    // the bin's counters are not read again: clear them for the next call
    // (the per-filament kernel counts into them)
    if (threadIdx.x == 0) {
        S.cnt[a][b] = 0;
        S.fill[a][b] = 0;
    }
    rank_sort_bin<kSortLds>(S.perm[a], S.key[a], s, n, v);
}

// sorted copies for the spread (by tile) and the pairs (by cell), one pass;
// thread (p, d) handles axis d of sorted entry p (its stencil base and w
// kernel values, and component d of the charges and pair position).  A
// separate launch from the per-bin sort: there a heavy bin's workgroup would
// gather its entries alone (measured 5.5 + 6.4 us -> 21.6 us fused).
struct GatherOut {
    int4 *base;
    void *ker, *q, *schg;
    double4 *spos;   // w: the point's segment index
};

// (the w kernel values of thread t go to lk[0 .. w-1]; the caller writes them
// to ker[t w ..])
template <typename R>
__device__ __forceinline__ void gather_one(int t, int w, int Q, const int *__restrict__ sperm,
                                           const int *__restrict__ pperm,
                                           const double *__restrict__ pos,
                                           const double *__restrict__ chg, double L, double inv_h,
                                           int n, double zeta, double inv_den, const GatherOut &G,
                                           R *lk) {
    const int p = t / 3, d = t - 3 * p;
    R *q = (R *)G.q, *schg = (R *)G.schg;
    int o = sperm[p];
    double f;
    const int b = stencil_base(wrap_box(pos[3 * o + d], L), inv_h, w, n, &f);
    const double half = 0.5 * w;
    for (int k = 0; k < w; k++) lk[k] = (R)kb_phi((k - f) / half, zeta, inv_den);
    int *bp = (int *)(G.base + p);
    bp[d] = b;
    q[4 * (size_t)p + d] = (R)chg[3 * o + d];
    o = pperm[p];
    double *sp = (double *)(G.spos + p);
    sp[d] = wrap_box(pos[3 * o + d], L);
    schg[4 * (size_t)p + d] = (R)chg[3 * o + d];
    if (d == 0) {
        bp[3] = 0;
        q[4 * (size_t)p + 3] = (R)0;
        sp[3] = (double)(o / Q);
        schg[4 * (size_t)p + 3] = (R)0;
    }
}

// Thread t = 3 p + d writes its kernel values at ker[t w ..], so those of a
// workgroup form one contiguous range: they are staged in LDS and written out
// with consecutive threads on consecutive words (a thread writing its own w
// values touched a cache line per lane in each store).  256 threads, w <= 16.
constexpr int kGatherBlock = 256;
template <typename R>
__global__ __launch_bounds__(kGatherBlock) void k_gather_all(int M, int w, int Q,
                                                             const int *__restrict__ sperm,
                                                             const int *__restrict__ pperm,
                                                             const double *__restrict__ pos,
                                                             const double *__restrict__ chg,
                                                             double L, double inv_h, int n,
                                                             double zeta, double inv_den,
                                                             GatherOut G) {
    __shared__ R lk[kGatherBlock * 16];
    const int t0 = blockIdx.x * kGatherBlock, t = t0 + (int)threadIdx.x;
    if (t0 >= 3 * M) return;   // uniform over the workgroup
    if (t < 3 * M)
        gather_one<R>(t, w, Q, sperm, pperm, pos, chg, L, inv_h, n, zeta, inv_den, G,
                      lk + threadIdx.x * w);
    __syncthreads();
    const int nt = 3 * M - t0 < kGatherBlock ? 3 * M - t0 : kGatherBlock;
    R *ker = (R *)G.ker + (size_t)t0 * w;
    for (int i = threadIdx.x; i < nt * w; i += kGatherBlock) ker[i] = lk[i];
}

void build_bins(bs_plan_t p) {
    const int bs = 256;
    const int M = (int)p->Nq, N = (int)p->N;
    const double L = p->prm.L, inv_h = p->n / L;
    const int w = p->prm.w, n = p->n;
    const int ntiles = p->NT * p->NT * p->NT, nc3 = p->nc * p->nc * p->nc;
    SortSet S;
    S.key[0] = (int *)p->sp_key.p; S.cnt[0] = (int *)p->sp_cnt.p; S.start[0] = (int *)p->sp_start.p;
    S.fill[0] = (int *)p->sp_fill.p; S.perm[0] = (int *)p->sp_perm.p;
    S.key[1] = (int *)p->pq_key.p; S.cnt[1] = (int *)p->pq_cnt.p; S.start[1] = (int *)p->pq_start.p;
    S.fill[1] = (int *)p->pq_fill.p; S.perm[1] = (int *)p->pq_perm.p;
    S.key[2] = (int *)p->nd_key.p; S.cnt[2] = (int *)p->nd_cnt.p; S.start[2] = (int *)p->nd_start.p;
    S.fill[2] = (int *)p->nd_fill.p; S.perm[2] = (int *)p->nd_perm.p;
    S.nbins[0] = ntiles; S.nbins[1] = nc3; S.nbins[2] = nc3;
    S.nitems[0] = M; S.nitems[1] = M; S.nitems[2] = N;
    const int maxb = ntiles > nc3 ? ntiles : nc3;
    const double zeta = p->prm.zeta, inv_den = 1.0 / (-expm1(-2.0 * zeta));
    GatherOut G;
    G.base = (int4 *)p->sp_base.p;
    G.ker = p->sp_ker.p;
    G.q = p->sp_q.p;
    G.spos = (double4 *)p->pq_pos.p;
    G.schg = p->pq_chg.p;
    const double *qp = (const double *)p->d_qpos.p, *qc = (const double *)p->d_qchg.p;
    // keys and counts come from the per-filament kernel (bin_keys)
    if (maxb <= (1 << 16)) {
        hipLaunchKernelGGL(k_scan_small, dim3(3), dim3(1024), 0, p->stream, S);
    } else {
        for (int a = 0; a < 3; a++)
            exclusive_scan(p, S.cnt[a], S.start[a], S.nbins[a], (int *)p->red_tmp.p);
    }
    hipLaunchKernelGGL(k_scatter_all, dim3(ceil_div(2 * M + N, bs)), dim3(bs), 0, p->stream, S);
    hipLaunchKernelGGL(k_sort_all, dim3(ntiles + 2 * nc3), dim3(64), 0, p->stream, S);
    if (p->fp32)
        hipLaunchKernelGGL(k_gather_all<float>, dim3(ceil_div(3 * (int64_t)M, kGatherBlock)),
                           dim3(kGatherBlock), 0,
                           p->stream, M, w, p->Q, S.perm[0], S.perm[1], qp, qc, L, inv_h, n, zeta,
                           inv_den, G);
    else
        hipLaunchKernelGGL(k_gather_all<double>, dim3(ceil_div(3 * (int64_t)M, kGatherBlock)),
                           dim3(kGatherBlock), 0,
                           p->stream, M, w, p->Q, S.perm[0], S.perm[1], qp, qc, L, inv_h, n, zeta,
                           inv_den, G);
}

BinKeys bin_keys(bs_plan_t p) {
    BinKeys k;
    k.key[0] = (int *)p->sp_key.p; k.cnt[0] = (int *)p->sp_cnt.p;
    k.key[1] = (int *)p->pq_key.p; k.cnt[1] = (int *)p->pq_cnt.p;
    k.key[2] = (int *)p->nd_key.p; k.cnt[2] = (int *)p->nd_cnt.p;
    k.L = p->prm.L;
    k.inv_h = p->n / p->prm.L;
    k.w = p->prm.w; k.n = p->n; k.T = p->T; k.NT = p->NT; k.nc = p->nc;
    return k;
}

}  // namespace bs
