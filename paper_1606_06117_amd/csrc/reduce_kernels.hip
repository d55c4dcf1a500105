// Reductions: FP64 error/mass sums and the FP32 velocity maximum.
//
// Both are two-level trees with a fixed number of blocks and a fixed
// per-thread stride, so a result depends only on the element count, never
// on the device, on timing or on the alignment of the inputs: bitwise
// reproducible.

#include "common.h"

namespace sla {
namespace {

constexpr int kThreads = 256;

// NaN-propagating maximum.
__device__ __forceinline__ double max_nan(double m, double v) { return (v > m || v != v) ? v : m; }
__device__ __forceinline__ float max_nan(float m, float v) { return (v > m || v != v) ? v : m; }

// Per block: partial sums of (a-b)^2, b^2, max|a-b|, a, b over a grid-stride
// range of groups of four elements; the block's 256 partials are combined
// in a fixed tree.  VEC: both arrays 16-byte aligned, a group is one load
// per array; otherwise four.  The n % 4 tail elements go to the first
// threads.
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_norms_part(int64_t n, const float* __restrict__ a,
                                                         const float* __restrict__ b,
                                                         double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0, mx = 0.0, sa = 0.0, sb = 0.0;
  auto add = [&](double va, double vb) {
    const double d = va - vb;
    s0 = fma(d, d, s0);
    s1 = fma(vb, vb, s1);
    mx = max_nan(mx, fabs(d));
    sa += va;
    sb += vb;
  };
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  // Both forms give every thread the same groups of four consecutive
  // elements in the same order, so the result does not depend on the
  // alignment of a and b.
  const int64_t n4 = n / 4;
  for (int64_t i = gid; i < n4; i += stride) {
    float4 va, vb;
    if (VEC) {
      va = reinterpret_cast<const float4*>(a)[i];
      vb = reinterpret_cast<const float4*>(b)[i];
    } else {
      va = make_float4(a[4 * i], a[4 * i + 1], a[4 * i + 2], a[4 * i + 3]);
      vb = make_float4(b[4 * i], b[4 * i + 1], b[4 * i + 2], b[4 * i + 3]);
    }
    add(va.x, vb.x);
    add(va.y, vb.y);
    add(va.z, vb.z);
    add(va.w, vb.w);
  }
  if (gid < n - 4 * n4) add(a[4 * n4 + gid], b[4 * n4 + gid]);
  __shared__ double sh[5][kThreads];
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = mx;
  sh[3][threadIdx.x] = sa;
  sh[4][threadIdx.x] = sb;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      const int j = threadIdx.x + w;
      sh[0][threadIdx.x] += sh[0][j];
      sh[1][threadIdx.x] += sh[1][j];
      sh[2][threadIdx.x] = max_nan(sh[2][threadIdx.x], sh[2][j]);
      sh[3][threadIdx.x] += sh[3][j];
      sh[4][threadIdx.x] += sh[4][j];
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) part[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

// One block: combine nblk partials in a fixed order.
__global__ __launch_bounds__(kThreads) void k_norms_final(int nblk, const double* __restrict__ part,
                                                          double* __restrict__ out5) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += kThreads) {
    v[0] += part[i * 5 + 0];
    v[1] += part[i * 5 + 1];
    v[2] = max_nan(v[2], part[i * 5 + 2]);
    v[3] += part[i * 5 + 3];
    v[4] += part[i * 5 + 4];
  }
  __shared__ double sh[5][kThreads];
  for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      const int j = threadIdx.x + w;
      sh[0][threadIdx.x] += sh[0][j];
      sh[1][threadIdx.x] += sh[1][j];
      sh[2][threadIdx.x] = max_nan(sh[2][threadIdx.x], sh[2][j]);
      sh[3][threadIdx.x] += sh[3][j];
      sh[4][threadIdx.x] += sh[4][j];
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) out5[threadIdx.x] = sh[threadIdx.x][0];
}

// Max |u_d| over the grid for each of ndim planes: blockIdx.y = axis.
// VEC: every plane starts on a 16-byte boundary (aligned u, ncells a
// multiple of 4): four values per load.  The maximum does not depend on the
// order, so both forms give the same result.
template <bool VEC>
__global__ __launch_bounds__(kThreads) void k_umax_part(int ncells, const float* __restrict__ u,
                                                        float* __restrict__ part) {
  const float* p = u + (size_t)blockIdx.y * ncells;
  float m = 0.f;
  const int stride = gridDim.x * kThreads;
  if (VEC) {
    const float4* p4 = reinterpret_cast<const float4*>(p);
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < ncells / 4; i += stride) {
      const float4 v = p4[i];
      m = max_nan(max_nan(m, fabsf(v.x)), fabsf(v.y));
      m = max_nan(max_nan(m, fabsf(v.z)), fabsf(v.w));
    }
  } else {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < ncells; i += stride)
      m = max_nan(m, fabsf(p[i]));
  }
  __shared__ float sh[kThreads];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = max_nan(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kThreads) void k_umax_final(int nblk, const float* __restrict__ part,
                                                         float* __restrict__ out) {
  const float* p = part + (size_t)blockIdx.x * nblk;
  float m = 0.f;
  for (int i = threadIdx.x; i < nblk; i += kThreads) m = max_nan(m, p[i]);
  __shared__ float sh[kThreads];
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) sh[threadIdx.x] = max_nan(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

}  // namespace

hipError_t launch_norms(int64_t n, const float* a, const float* b, double* part, double* out5,
                        hipStream_t st) {
  const bool vec = (reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(k_norms_part<true>, dim3(kNormBlocks), dim3(kThreads), 0, st, n, a, b, part);
  else
    hipLaunchKernelGGL(k_norms_part<false>, dim3(kNormBlocks), dim3(kThreads), 0, st, n, a, b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(kThreads), 0, st, kNormBlocks, part, out5);
  return hipGetLastError();
}

hipError_t launch_umax(int ndim, int ncells, const float* u, float* part, float* out3,
                       hipStream_t st) {
  if (reinterpret_cast<uintptr_t>(u) % 16 == 0 && ncells % 4 == 0)
    hipLaunchKernelGGL(k_umax_part<true>, dim3(kUmaxBlocks, ndim), dim3(kThreads), 0, st, ncells, u,
                       part);
  else
    hipLaunchKernelGGL(k_umax_part<false>, dim3(kUmaxBlocks, ndim), dim3(kThreads), 0, st, ncells, u,
                       part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_umax_final, dim3(ndim), dim3(kThreads), 0, st, kUmaxBlocks, part, out3);
  return hipGetLastError();
}

}  // namespace sla
