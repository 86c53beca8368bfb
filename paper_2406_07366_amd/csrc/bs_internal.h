// Internal declarations of libbs.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bs.h"

namespace bs {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kMaxQ = 4;
// nodes per filament whose spline solve stays in LDS (cubic, quintic);
// longer filaments use the plan's global scratch
constexpr int kPcrLds = 128;
constexpr int kPcr5Lds = 64;
constexpr int kMinW = 4, kMaxW = 16;

// Gauss-Legendre nodes h_i in [0,1] and weights w_i (sum 1) for Q = 1..4.
struct GLRule {
    double h[kMaxQ];
    double w[kMaxQ];
};
GLRule gl_rule(int Q);

// Growable device buffer.
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Geometry;  // device views, see geometry.hip

}  // namespace bs

struct bs_plan_s {
    bs_params prm{};        // resolved parameters
    hipStream_t stream = nullptr;
    // side stream (default priority): the short-range sum and the
    // near-singular correction of bs_velocity run there, concurrently with
    // the long-range chain on the plan stream; fork and join by events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the near-singular pair search of bs_set_filaments also runs on the side
    // stream (beside the velocity's long-range stages); until a later call
    // joins the side stream back, side_pending is set and ev_ns marks the
    // search's end
    hipEvent_t ev_ns = nullptr;
    bool side_pending = false;
    int device = 0;
    std::string err;
    int fp32 = 0;           // precision == BS_FP32_MIXED
    size_t real_size = 8;   // bytes of a grid real

    // grid and FFT
    int n = 0;              // grid points per axis
    int T = 8;              // spread tile edge (cells)
    int NT = 0;             // tiles per axis
    hipfftHandle fft_fwd = 0, fft_inv = 0;
    bs::DBuf grid;          // [3][n][n][n] real
    bs::DBuf spec;          // [3][n][n][n/2+1] complex
    bs::DBuf deconv;        // [K+1] float64: 1 / F(m)^2 per axis
    bs::DBuf fftwork;
    // pruned transforms (power-of-two grids): twiddles [n forward][n
    // inverse], A [3][n][n][K+1] and B [3][2K+1][n][K+1] complex; batch sizes
    bool pruned = false;
    int fft_rb = 1, fft_kb = 1, fft_kz = 1;
    bs::DBuf fft_tw, fft_A, fft_B;

    // short-range cell list
    int nc = 1;             // cells per axis

    // filaments
    int64_t nfil = 0, N = 0, Nq = 0;
    int Q = 2;
    int order = 4;          // spline order: 4 cubic, 6 quintic
    std::vector<int64_t> off_host;
    bool have_filaments = false;
    bs::DBuf d_off, d_fil, d_gamma;            // int32 [nfil+1], int32 [N], f64 [nfil]
    bs::DBuf d_x;                              // f64 [N][3] private copy of nodes
    bs::DBuf d_xn;                             // f64 [N][3] end node of segment j in
                                               // j's frame (next node, plus the
                                               // filament's period shift after the
                                               // last node of an infinite filament)
    bs::DBuf d_shift;                          // f64 [nfil][3] period shifts n_l L
    int64_t nper = 0;                          // filaments the shifts were set for
    bs::DBuf d_dtau, d_D, d_sdd, d_ell;        // node geometry
    bs::DBuf d_qpos, d_qchg;                   // f64 [Nq][3]
    bs::DBuf d_status;                         // int32 device status word
    // spread binning
    bs::DBuf sp_key, sp_cnt, sp_start, sp_fill, sp_perm;
    bs::DBuf sp_base, sp_ker, sp_q;
    // pair binning
    bs::DBuf pq_key, pq_cnt, pq_start, pq_fill, pq_perm;
    bs::DBuf pq_pos, pq_chg;                   // double4 (position, segment), charges
    bs::DBuf nd_key, nd_cnt, nd_start, nd_fill, nd_perm;
    // scan scratch, reductions, spline scratch (filaments over 512 nodes)
    bs::DBuf scan_tmp, red_tmp, spline_tmp;
    int64_t max_fil_nodes = 0;
    // near-singular pairs
    int ns_max_per_node = 64;                  // near-singular segments per target, at most
    int ns_ncmax = 3;                          // bound on the segment cell grid per axis
    bs::DBuf ns_red, ns_nc;                    // f64 [1 + blocks] max reach, int32 cells per axis
    bs::DBuf ns_ckey, ns_ccnt, ns_cstart, ns_cfill, ns_cperm;   // segments by midpoint cell
    bs::DBuf ns_tkey, ns_tcnt, ns_tstart, ns_tfill, ns_tperm;   // targets by node cell
    bs::DBuf ns_segA, ns_segB;                 // double4 [N] cell-ordered end points
    bs::DBuf ns_segM, ns_segH;                 // float4 [N] flag-test capsules (midpoint,
                                               // eta ell; half chord, periods)
    bs::DBuf ns_slots;                         // int2 [N][max_per_node] per-node flag output
    bs::DBuf ns_cnt, ns_start, ns_pairs, ns_pnode, ns_pout;
    // learned correction
    bs_mlp_t mlp = nullptr;
    float ns_err[16] = {};
    bs::DBuf ns_X, ns_Y;                       // features, outputs of the learned pairs
    bs::DBuf ns_fallback;                      // int32 [4]: learned pairs, plain-integrator pairs,
                                               // gate open, gate closed (set on the device)
    bs::DBuf ns_learn;                         // int32 [pairs]: pairs the network takes
    bs::DBuf ns_fblist;                        // int32 [pairs]: pairs the learned
                                               // path hands to the graded panels
    bs::DBuf ns_vs;                            // f64 [1 + blocks]: velocity scale
    // RK4 stage buffers
    bs::DBuf rk_k, rk_s;
    // graph replay of bs_step
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *g_xyz = nullptr, *g_gamma = nullptr;
    double *g_v = nullptr;
    // terms (for velocity terms / energy)
    bs::DBuf tmp3;                             // f64 [N][3]
    bs::DBuf e_D, e_S;                         // f64 [N][3]: spline of psi (energy)
    bs::DBuf d_vls;                            // f64 [N][3]: local - self velocity
    // per-stage timing (diagnostics)
    bool prof = false;
    hipEvent_t ev_beg[BS_NSTAGES] = {}, ev_end[BS_NSTAGES] = {};
    bool ev_used[BS_NSTAGES] = {};
    double stage_ms[BS_NSTAGES] = {};
    int64_t stage_cnt[BS_NSTAGES] = {};
};

namespace bs {

int set_error(bs_plan_t p, int code, const std::string &msg);
int check_hip(bs_plan_t p, hipError_t e, const char *what);

// geometry.hip
// chord lengths, spline, quadrature points, charges, segment lengths and the
// velocity's local-minus-self term (d_vls), one workgroup per filament
void launch_filaments(bs_plan_t p, const double *xyz, const double *gamma);
// spline through periodic nodal data (such as the streamfunction) on the
// plan's knots: slopes (and, quintic, second derivatives) into Dout, Sout
void launch_spline_data(bs_plan_t p, const double *data, double *Dout, double *Sout);
// mode bits for launch_local_self
enum { LS_VLOCAL = 1, LS_VSELF = 2, LS_PSI = 4, LS_ASSIGN = 8 };
void launch_local_self(bs_plan_t p, int mode, double sign, double *out);

// binning.hip
void exclusive_scan(bs_plan_t p, const int *in, int *out, int n, int *sums);
void build_bins(bs_plan_t p);
// what the per-filament kernel needs to key and count the three bin sorts
// (quadrature points by spread tile and by pair cell, nodes by pair cell);
// the counters start at zero (cleared at allocation, and by the per-bin sort
// of the previous call)
struct BinKeys {
    int *key[3], *cnt[3];
    double L, inv_h;
    int w, n, T, NT, nc;
};
BinKeys bin_keys(bs_plan_t p);

// nufft.hip
void launch_spread(bs_plan_t p);
void launch_spectral(bs_plan_t p, int psi);
// out = base + interpolated long-range term (base NULL: out += ...)
void launch_interp(bs_plan_t p, const double *base, double *out);
void launch_modes(bs_plan_t p, double *out);
int fft_forward(bs_plan_t p);
int fft_inverse(bs_plan_t p);

// fft.hip
bool pruned_fft_ok(int n, size_t csize);
void pruned_batches(int n, size_t csize, int *rb, int *kb, int *kz);
void pruned_forward(bs_plan_t p);
void pruned_spectral_op(bs_plan_t p, int psi);
void pruned_inverse(bs_plan_t p);
// the inverse transforms leave the grid [n][n][n][3] (components interleaved)
// rather than [3][n][n][n]: the pruned path on grids above 64^3
bool grid_interleaved(bs_plan_t p);

// pairs.hip
// out = base + short-range term (base NULL: out += short-range term);
// alone: nothing else runs beside it (more wavefronts per target on small
// inputs)
void launch_pairs(bs_plan_t p, int psi, const double *base, double *out, bool alone);

// ns.hip
void ns_build_pairs(bs_plan_t p);
// v += near-singular correction (graded panels / mapped rule / learned with
// the graded panels where its indicator refuses; base: the array whose rms
// over the nodes is the learned path's velocity scale)
void launch_ns_adaptive(bs_plan_t p, double *v);
void launch_ns_mapped(bs_plan_t p, double *v);
void launch_ns_mlp(bs_plan_t p, double *v, const double *base);
// mlp.hip: inference with the sample count read on the device
void mlp_forward_device(bs_mlp_t m, const int *Bdev, int64_t Bmax, const float *X, float *Y,
                        hipStream_t stream);
hipStream_t mlp_stream(bs_mlp_t m);

// pairs.hip (with the short-range sums): the energy line integral
void launch_energy(bs_plan_t p, const double *psi, double *partial, int nblocks);

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// stage timing: record begin/end events on the plan stream when profiling
inline void stage_begin(bs_plan_t p, int s) {
    if (p->prof) { (void)hipEventRecord(p->ev_beg[s], p->stream); p->ev_used[s] = true; }
}
inline void stage_end(bs_plan_t p, int s) {
    if (p->prof) (void)hipEventRecord(p->ev_end[s], p->stream);
}
void stage_collect(bs_plan_t p);

}  // namespace bs
