// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sla {

enum { CIR = 0, FEC = 1, BEC = 2, CEC = 3, CEC_LITERAL = 4 };  // CEC_LITERAL: sweep combination only

// Grid geometry as the kernels see it.  lam[d] = fl32(dt / dx[d]); unused
// axes have n = 1 and lam = 0.
struct Geo {
  int nx, ny, nz;
  int ncells;
  float lam[3];
};

// Kernels that address a field by 32-bit byte offsets from a row or plane
// start (the fused step, the marching sweeps): every offset + 4 stays below
// 2^32 for fields of fewer than 2^30 cells, and of exactly 2^30 cells when
// ny >= 2 (an offset then spans at most the field minus one row).
inline bool offsets32_ok(const Geo& g) {
  const size_t n = (size_t)g.ncells, lim = size_t(1) << 30;
  return n < lim || (n == lim && g.ny >= 2);
}

// Reach (halo in cells) each kernel serves, one per axis: reach[d] =
// floor(max |c_d|) + 1, at most SLA_MAX_REACH.
struct Reach {
  int r[3];
};

// ---------------------------------------------------------------- launchers
// All launchers return hipSuccess or the error of the launch.  `flag` is a
// device int set to 1 by a kernel that had to clamp a backtrace offset.

hipError_t launch_cir(int ndim, const Geo& g, const float* phi, const float* u,
                      float* out, int* flag, hipStream_t st);

// Unsplit fused FEC or BEC step (scheme = FEC or BEC), reach R (max over axes).
hipError_t launch_ec(int ndim, int scheme, int R, const Geo& g, const float* phi,
                     const float* u, float* out, int* flag, hipStream_t st);

// Unsplit FEC or BEC step of a 3D grid at reach 1, all calls in one pass
// (a z-march with every stage's field in LDS); needs offsets32_ok(g).  Same
// results as the chain of gather kernels.
hipError_t launch_ec_march(int scheme, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, int shape = 0);

// One third-order sweep along axis d with reach R; u_d is that axis' plane.
// march: y and z sweeps of grids of at most 2^30 cells walk columns through
// registers (k_sweep_m); otherwise LDS tiles (k_sweep_s).  Same results.
// One gather call of the chained unsplit FEC / BEC: mode 1 writes
// a + (b - L_{-U}[a])/2 (FEC's result, a = Phi1, b = Phi), mode 2
// b + (b - L_{-U}[a])/2 (BEC's psi).  out may equal b.
hipError_t launch_ec_gather(int ndim, int mode, const Geo& g, const float* a, const float* b,
                            const float* u, float* out, int* flag, hipStream_t st);
// One FEC (scheme FEC), BEC (scheme BEC) or literal large-CFL third-order
// (scheme CEC_LITERAL) sweep along axis d: the one-dimensional scheme
// applied along one axis, reach 1-4, by the kernels of launch_cec_sweep
// (march: window and marching sweeps; otherwise LDS tiles).
hipError_t launch_ec_sweep(int scheme, int d, int R, const Geo& g, const float* phi,
                           const float* ud, float* out, int* flag, hipStream_t st, bool march);
// One third-order sweep along axis d with a midpoint backtrace: the calls of
// L_U depart from x - c(x - c/2), the call of L_{-U} from x + c(x + c/2)
// (tile kernels, reach 1-4).
hipError_t launch_cec_sweep_mid(int d, int R, const Geo& g, const float* phi, const float* ud,
                                float* out, int* flag, hipStream_t st);
hipError_t launch_cec_sweep(int d, int R, const Geo& g, const float* phi,
                            const float* u_d, float* out, int* flag, hipStream_t st,
                            bool march = true);
// The x and y sweeps of a split step in one kernel: x then y if xfirst,
// else y then x; u holds the x and y planes.  scheme: the third order (CEC),
// FEC, BEC or CEC_LITERAL along each axis.  Same results as the two sweeps.
// pairs: two nodes per lane, even nx, reach R <= 3 on both axes; otherwise
// one node per lane, R <= 2.  Needs offsets32_ok(g).
hipError_t launch_cec_sweep_xy(int R, bool xfirst, const Geo& g, const float* phi, const float* u,
                               float* out, int* flag, hipStream_t st, bool pairs, int scheme = CEC);

// Fused three-axis third-order step (reach 1 only): x,y,z order if even,
// z,y,x otherwise.  variant: 1 register segments, 2 streaming (direct
// global-to-LDS loads), 4 window march with 4-row segments (no LDS), 5 the
// fastest of these per parity and grid size, 6 window march with 8-row
// segments, 7 window march whose workgroups share segment halos through
// LDS, 8 the same with 16-row groups of 12 waves, in march chunks or
// persistent, 9 as 8 with the inputs loaded two planes ahead, 10-13 as 8
// and 9 with one or two windows per workgroup, 14 the march on aligned
// 128-node windows of two nodes per lane; all perform the same FP32
// operations (0 and 3 are unused).
constexpr int kCec3dVariants = 15;
inline bool cec3d_variant_ok(int v) { return v >= 1 && v < kCec3dVariants && v != 3; }
// Launch shape: y planes per workgroup, or for variant 8 the march chunk
// (< 0: -chunk planes) or workgroups per CU of the persistent form (> 0);
// 0: the default for the grid; and whether tiles are mapped to XCDs in
// contiguous ranges (1) or round robin.
struct Cec3dLaunch {
  int ychunk = 0;
  int swizzle = 1;
};
int cec3d_default_ychunk(const Geo& g);
// The fused step of k = 1, 2 or 4 fields sharing the velocity u (reach 1):
// in[f] -> out[f]; the velocity is loaded once per tile for the k fields.
// Every field's result equals launch_cec3d's bit for bit.  chunk: march
// planes per workgroup (0: the default).
hipError_t launch_cec3d_multi(int k, bool even, const Geo& g, const float* const* in,
                              float* const* out, const float* u, int* flag, hipStream_t st,
                              int chunk = 0);
hipError_t launch_cec3d(int variant, bool even, const Geo& g, const float* phi, const float* u,
                        float* out, int* flag, hipStream_t st, Cec3dLaunch lc = Cec3dLaunch());

// ---------------------------------------------------------------- network
constexpr int kMlpInputs = 32;   // 27 differences + 3 Courant numbers + 2 zero
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpInputs * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;
constexpr int kMlpMaxBlocks = 512;  // training blocks (gradient partials)
// floats per block of gradient partials (whole 16-byte groups)
constexpr int kMlpPartStride = (kMlpParams + 3) / 4 * 4;
constexpr int kLearnedBlocks = 1024;  // workgroups of a learned-step launch (each loads the weights once)
constexpr int kMlpPackElems = kMlpHidden * kMlpInputs + 2 * kMlpHidden * kMlpHidden;

size_t mlp_train_lds();
// Forward (and, if train, backward) over m feature rows; nblk_out receives
// the number of gradient partials written.
hipError_t launch_mlp(bool train, const void* X, const float* target, int m, float inv_m2,
                      const void* wpack, const float* wr, float* yout, float* gpart,
                      float* lpart, int* nblk_out, hipStream_t st);
hipError_t launch_grad_reduce(const float* gpart, const float* lpart, int nblk, float* grad,
                              double* loss_sum, hipStream_t st);
// launch_grad_reduce with the training step's Adam update of every parameter
// (Adam, Kingma & Ba, on the FP32 master weights) in the same kernel.
hipError_t launch_grad_adam(const float* gpart, const float* lpart, int nblk, float* grad,
                            double* loss_sum, float* master, float* m, float* v, float lr,
                            float beta1, float beta2, float eps, float bc1, float bc2, float* wr,
                            void* wpack, hipStream_t st);
hipError_t launch_pack(const float* master, float* wr, void* wpack, hipStream_t st);
hipError_t launch_make_pairs(const Geo& g, const float* phi1, const float* phi_next, const float* u,
                             const int* cells, int m, void* X, float* target, float* sigma,
                             hipStream_t st);
hipError_t launch_learned_correct(const Geo& g, const float* phi1, const float* u, const void* wpack,
                                  const float* wr, float* out, hipStream_t st);
// The same correction as a march along z (LDS-staged neighbourhoods, one
// node per lane for the features); same results bit for bit.
hipError_t launch_learned_march(const Geo& g, const float* phi1, const float* u, const void* wpack,
                                const float* wr, float* out, hipStream_t st);

// Segment variant of the same step (identical arithmetic per node).
hipError_t launch_cec3d_seg(bool even, const Geo& g, const float* phi, const float* u, float* out,
                            int* flag, hipStream_t st, Cec3dLaunch lc = Cec3dLaunch());

// Streaming variant (direct global-to-LDS loads, 512-thread workgroups).
hipError_t launch_cec3d_v4(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc = Cec3dLaunch());

// One problem of a batched step.  buf[parity] is read and buf[parity ^ 1]
// written; u are velocity planes (umask ~0u) or three single values of a
// uniform velocity (umask 0).  Tiles are 64 (x) x 16 (z) x ychunk (y).
struct BatchProblem {
  float* buf[2];
  const float* u[3];
  unsigned umask;
  int n[3];
  float lam[3];
  int ychunk;
};
constexpr int kBatchTileX = 64, kBatchTileZ = 16;
hipError_t launch_cec3d_batch(bool even, const BatchProblem* probs, const int4* items, int nitems,
                              int parity, int grid, int* flag, hipStream_t st);
int cec3d_batch_blocks_per_cu();
hipError_t launch_batch_copy_back(const BatchProblem* probs, int nprob, hipStream_t st);

// Max |u_d| per axis over the grid (FP32, NaN propagates) into out3 (device).
hipError_t launch_umax(int ndim, int ncells, const float* u, float* part,
                       float* out3, hipStream_t st);
constexpr int kUmaxBlocks = 512;

// FP64 reductions {sum (a-b)^2, sum b^2, max|a-b|, sum a, sum b} into out5
// (device).  part holds kNormBlocks*5 doubles.
hipError_t launch_norms(int64_t n, const float* a, const float* b, double* part,
                        double* out5, hipStream_t st);
constexpr int kNormBlocks = 1024;

}  // namespace sla
