// Fused third-order 3D step: all three axis sweeps of one time step in one
// pass over HBM (read phi and u once, write phi once: 20 B per cell).
//
// What is computed is the per-axis third-order sweep (eq. intro:CEC with the
// weights of eq. intro:CECcoef, one axis at a time as in eqs. split:1-2),
// applied x, y, z on even steps and z, y, x on odd steps.  Per axis and node:
//   Phi1 = L_U Phi,  e = Phi - L_{-U} Phi1,
//   out  = Phi1 + 1/2 [e_a + (1+f)/3 (e_b - e_a)].
//
// Layout of the work.  A workgroup owns an x-z tile of TX x TZ cells and
// marches along y over a chunk of planes.  The middle sweep (y) is then a
// pipeline along the march: each thread keeps, for its columns, rings of the
// last three planes of its input, Phi1 and e in registers, so the y halo
// costs a pipeline delay and no recomputation.  The first sweep (x on even
// steps, z on odd ones) runs in-plane through LDS on the tile grown by the
// last sweep's halo; the last sweep (z, resp. x) runs in-plane on the y
// output.  Both orders share this kernel with the roles of x and z swapped.
//
// This kernel serves reach 1 (every |c| < 1): the departure interval of a
// node is (i, i - s) and each call reads one neighbour.

#include <type_traits>

#include "common.h"

namespace sla {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

// Reach-1 departure: fraction and far-node offset (+-1) for c and for -c.
struct Dep1 {
  float f;
  int ob;   // far node of L_U:    i + ob, ob = -1 if c >= 0 else +1
  int obr;  // far node of L_{-U}: i + obr, obr = -1 if -c >= 0 else +1
};

__device__ __forceinline__ Dep1 depart1(float c, int* flag) {
  const float mag = fabsf(c);
  float f = mag;
  if (!(mag < 1.f)) {  // beyond reach 1: keep the fraction, record it
    if (mag == mag) *flag = 1;
    f = mag - floorf(mag);
  }
  Dep1 d;
  d.f = f;
  d.ob = c >= 0.f ? -1 : 1;
  d.obr = c > 0.f ? 1 : -1;
  return d;
}

template <bool EVEN>
struct Cec3dShape {
  static constexpr int R = 1;
  static constexpr int H = 3 * R;      // halo of a sweep's input
  static constexpr int TX = 64, TZ = 16;
  static constexpr int W = TX + 2 * H; // padded row length (x)
  static constexpr int HZ = TZ + 2 * H;
  static constexpr int NP = W * HZ;    // padded plane
  static constexpr int KP = (NP + kThreads - 1) / kThreads;  // padded-plane cells per thread
  // first sweep along A, last along B
  static constexpr int TA = EVEN ? TX : TZ;
  static constexpr int TB = EVEN ? TZ : TX;
  static constexpr int SA = EVEN ? 1 : W;  // LDS stride along A
  static constexpr int SB = EVEN ? W : 1;  // LDS stride along B
  // y-pipeline region (A in [0, TA), B in [-H, TB + H)) as an x-fastest
  // rectangle [YX0, YX0 + YW) x [YZ0, YZ0 + YH)
  static constexpr int YX0 = EVEN ? 0 : -H;
  static constexpr int YW = EVEN ? TX : TX + 2 * H;
  static constexpr int YZ0 = EVEN ? -H : 0;
  static constexpr int YH = EVEN ? TZ + 2 * H : TZ;
  static constexpr int NY = YW * YH;
  static constexpr int KY = (NY + kThreads - 1) / kThreads;  // y columns per thread
};

// Run f(e) for e = tid + 256 k < N, unrolled so that the LDS reads of all of
// a thread's elements are issued before the first result is needed.
template <int N, typename F>
__device__ __forceinline__ void for_each_cell(F&& f) {
#pragma unroll
  for (int k = 0; k < (N + kThreads - 1) / kThreads; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (N % kThreads == 0 || e < N) f(e);
  }
}

// padded LDS index of tile-relative (x, z)
template <bool EVEN>
__device__ __forceinline__ int lidx(int x, int z) {
  using S = Cec3dShape<EVEN>;
  return (z + S::H) * S::W + (x + S::H);
}

// wrap a coordinate that is at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int v, int n) {
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

// Minimum waves per SIMD the compiler must leave room for (register budget).
#ifndef SLA_CEC3D_MIN_WAVES
#define SLA_CEC3D_MIN_WAVES 2
#endif

template <bool EVEN>
__global__ __launch_bounds__(kThreads, SLA_CEC3D_MIN_WAVES) void k_cec3d_r1(const float* __restrict__ phi,
                                                       const float* __restrict__ ux,
                                                       const float* __restrict__ uy,
                                                       const float* __restrict__ uz,
                                                       float* __restrict__ out, Geo g,
                                                       int ychunk, int* flag) {
  using S = Cec3dShape<EVEN>;
  constexpr int H = S::H, TA = S::TA, TB = S::TB, SA = S::SA, SB = S::SB;
  constexpr int KP = S::KP, KY = S::KY;
  __shared__ float P[S::NP];   // phi at the loaded plane, padded
  __shared__ float CA[S::NP];  // Courant numbers of the first sweep
  __shared__ float CB[S::NP];  // Courant numbers of the last sweep (output plane)
  __shared__ float S1[S::NP];  // Phi1 of the first, then of the last sweep
  __shared__ float SE[S::NP];  // e of the first, then of the last sweep
  __shared__ float AO[S::NP];  // first-sweep output (y-pipeline input)
  __shared__ float YO[S::NP];  // y-sweep output (last-sweep input)

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * S::TX, z0 = blockIdx.y * S::TZ;
  const int y0 = blockIdx.z * ychunk;
  const int y1 = min(y0 + ychunk, g.ny);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned nxy = unsigned(nx) * unsigned(ny);
  const float* uA = EVEN ? ux : uz;
  const float* uB = EVEN ? uz : ux;
  const float lamA = EVEN ? g.lam[0] : g.lam[2];
  const float lamB = EVEN ? g.lam[2] : g.lam[0];
  const float lamY = g.lam[1];

  // Per-thread global x-z offsets (the y term is added per plane), computed
  // once.  Padded plane: cell e = tid + 256 k; y region: x-fastest rectangle.
  unsigned poff[KP];
  unsigned yoff[KY];
  int ycol[KY];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int e = min(tid + k * kThreads, S::NP - 1);
    const int z = e / S::W - H, x = e % S::W - H;
    poff[k] = unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz));
  }
#pragma unroll
  for (int j = 0; j < KY; ++j) {
    const int e = min(tid + j * kThreads, S::NY - 1);
    const int z = S::YZ0 + e / S::YW, x = S::YX0 + e % S::YW;
    yoff[j] = unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz));
    ycol[j] = lidx<EVEN>(x, z);
  }
  auto pvalid = [&](int k) { return KP * kThreads == S::NP || tid + k * kThreads < S::NP; };
  auto yvalid = [&](int j) { return KY * kThreads == S::NY || tid + j * kThreads < S::NY; };

  // y-pipeline rings, per column: input a, Phi1, e, Courant (3 planes each)
  float ra[3][KY], r1[3][KY], re[3][KY], rc[3][KY];
#pragma unroll
  for (int j = 0; j < KY; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  // Register prefetch of the next plane: phi and the first sweep's velocity
  // (padded plane), the y velocity one plane back and the last sweep's
  // velocity at the next output plane (y region).
  float fp[KP], fa[KP], fy[KY], fb[KY];
  auto prefetch = [&](int t) {
    const unsigned qoff = unsigned(wrap1(y0 - H + t, ny)) * unsigned(nx);
    const unsigned coff = unsigned(wrap1(y0 - H + t - 1, ny)) * unsigned(nx);
    const unsigned ooff = unsigned(wrap1(y0 + t - 2 * H, ny)) * unsigned(nx);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      fp[k] = phi[poff[k] + qoff];
      fa[k] = uA[poff[k] + qoff];
    }
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      fy[j] = uy[yoff[j] + coff];
      fb[j] = uB[yoff[j] + ooff];
    }
  };

  const int iters = (y1 - y0) + 2 * H;
  prefetch(0);
  // The ring slot of local plane t is t % 3; the loop body is unrolled by 3
  // so that every slot index is a compile-time constant.
  auto body = [&](auto phase, int t) {
    constexpr int p0 = decltype(phase)::value;  // t % 3
    constexpr int p1 = (p0 + 2) % 3;            // (t - 1) % 3
    constexpr int p2 = (p0 + 1) % 3;            // (t - 2) % 3
    constexpr int p3 = p0;                      // (t - 3) % 3
    const bool emit = t >= 2 * H;

    // 1. publish the prefetched plane, then start fetching the next one
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (!pvalid(k)) continue;
      P[tid + k * kThreads] = fp[k];
      CA[tid + k * kThreads] = fa[k] * lamA;
    }
    float cy[KY];
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      cy[j] = fy[j] * lamY;
      if (emit && yvalid(j)) CB[ycol[j]] = fb[j] * lamB;
    }
    if (t + 1 < iters) prefetch(t + 1);
    __syncthreads();
    // 2. first sweep, Phi1 on A in [-2, TA+2)
    {
      constexpr int LA = TA + 4, LB = TB + 2 * H;
      for_each_cell<LA * LB>([&](int e) {
        const int b = -H + e / LA, a = -2 + e % LA;
        const int i = EVEN ? lidx<EVEN>(a, b) : lidx<EVEN>(b, a);
        const Dep1 d = depart1(CA[i], flag);
        S1[i] = lerp(P[i], P[i + d.ob * SA], d.f);
      });
    }
    __syncthreads();
    // 3. first sweep, e on A in [-1, TA+1)
    {
      constexpr int LA = TA + 2, LB = TB + 2 * H;
      for_each_cell<LA * LB>([&](int e) {
        const int b = -H + e / LA, a = -1 + e % LA;
        const int i = EVEN ? lidx<EVEN>(a, b) : lidx<EVEN>(b, a);
        const Dep1 d = depart1(CA[i], flag);
        SE[i] = P[i] - lerp(S1[i], S1[i + d.obr * SA], d.f);
      });
    }
    __syncthreads();
    // 4. first sweep output on A in [0, TA)
    {
      constexpr int LB = TB + 2 * H;
      for_each_cell<TA * LB>([&](int e) {
        const int b = -H + e / TA, a = e % TA;
        const int i = EVEN ? lidx<EVEN>(a, b) : lidx<EVEN>(b, a);
        const Dep1 d = depart1(CA[i], flag);
        const float ea = SE[i], eb = SE[i + d.ob * SA];
        const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
        AO[i] = fmaf(0.5f, fmaf(w, eb - ea, ea), S1[i]);
      });
    }
    __syncthreads();
    // 5. y sweep as a pipeline along the march (registers)
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      if (!yvalid(j)) continue;
      const int i = ycol[j];
      ra[p0][j] = AO[i];  // input at plane t
      rc[p1][j] = cy[j];  // Courant at plane t-1
      // Phi1 at plane t-1
      Dep1 d = depart1(rc[p1][j], flag);
      r1[p1][j] = lerp(ra[p1][j], d.ob < 0 ? ra[p2][j] : ra[p0][j], d.f);
      // e at plane t-2
      d = depart1(rc[p2][j], flag);
      re[p2][j] = ra[p2][j] - lerp(r1[p2][j], d.obr > 0 ? r1[p1][j] : r1[p3][j], d.f);
      // y-sweep output at plane t-3
      d = depart1(rc[p3][j], flag);
      const float ea = re[p3][j];
      const float eb = d.ob < 0 ? re[p1][j] : re[p2][j];  // e at t-4 (slot p1) or t-2
      const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
      YO[i] = fmaf(0.5f, fmaf(w, eb - ea, ea), r1[p3][j]);
    }
    __syncthreads();
    if (!emit) return;
    // 6. last sweep, Phi1 on B in [-2, TB+2)
    {
      constexpr int LB = TB + 4;
      for_each_cell<TA * LB>([&](int e) {
        const int b = -2 + e / TA, a = e % TA;
        const int i = EVEN ? lidx<EVEN>(a, b) : lidx<EVEN>(b, a);
        const Dep1 d = depart1(CB[i], flag);
        S1[i] = lerp(YO[i], YO[i + d.ob * SB], d.f);
      });
    }
    __syncthreads();
    // 7. last sweep, e on B in [-1, TB+1)
    {
      constexpr int LB = TB + 2;
      for_each_cell<TA * LB>([&](int e) {
        const int b = -1 + e / TA, a = e % TA;
        const int i = EVEN ? lidx<EVEN>(a, b) : lidx<EVEN>(b, a);
        const Dep1 d = depart1(CB[i], flag);
        SE[i] = YO[i] - lerp(S1[i], S1[i + d.obr * SB], d.f);
      });
    }
    __syncthreads();
    // 8. last sweep output on the tile, stored to HBM at plane t - 6
    {
      const unsigned yo = unsigned(y0 + t - 2 * H) * unsigned(nx);
      for_each_cell<TA * TB>([&](int e) {
        const int b = e / TA, a = e % TA;
        const int x = EVEN ? a : b, z = EVEN ? b : a;
        if (x0 + x >= nx || z0 + z >= nz) return;
        const int i = lidx<EVEN>(x, z);
        const Dep1 d = depart1(CB[i], flag);
        const float ea = SE[i], eb = SE[i + d.ob * SB];
        const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
        out[unsigned(x0 + x) + yo + nxy * unsigned(z0 + z)] =
            fmaf(0.5f, fmaf(w, eb - ea, ea), S1[i]);
      });
    }
    // The next plane stores CB before its first barrier while this plane's
    // last sweep may still be reading it.
    __syncthreads();
  };

  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
}

// ---------------------------------------------------------------------------
// Segment variant: the first and the last sweep of a plane run as per-thread
// segments of V consecutive nodes along the sweep axis, all three calls in
// registers (inputs V+6 nodes, Phi1 on V+4, e on V+2, outputs V), so a plane
// needs four barriers instead of seven.  The y pipeline is the same.
// ---------------------------------------------------------------------------
template <bool EVEN>
struct SegShape : Cec3dShape<EVEN> {
  using B = Cec3dShape<EVEN>;
  static constexpr int V = 8;
  static constexpr int NS1 = B::TA / V, N1 = (B::TB + 2 * B::H) * NS1;  // first sweep items
  static constexpr int NS2 = B::TB / V, N2 = B::TA * NS2;               // last sweep items
  static_assert(B::TA % V == 0 && B::TB % V == 0, "segments tile the block");
  static_assert(N1 <= kThreads && N2 <= kThreads, "one item per thread");
};

// Third-order sweep of one segment: p holds the V+6 input nodes a0-3..a0+V+2,
// c the V+4 Courant numbers of a0-2..a0+V+1; out receives a0..a0+V-1.
template <int V>
__device__ __forceinline__ void sweep_segment(const float (&p)[V + 6], const float (&c)[V + 4],
                                              float (&out)[V], int* flag) {
  float p1[V + 4], e[V + 2];
#pragma unroll
  for (int k = 0; k < V + 4; ++k) {  // node a0-2+k
    const Dep1 d = depart1(c[k], flag);
    p1[k] = lerp(p[k + 1], d.ob < 0 ? p[k] : p[k + 2], d.f);
  }
#pragma unroll
  for (int k = 0; k < V + 2; ++k) {  // node a0-1+k
    const Dep1 d = depart1(c[k + 1], flag);
    e[k] = p[k + 2] - lerp(p1[k + 1], d.obr > 0 ? p1[k + 2] : p1[k], d.f);
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {  // node a0+k
    const Dep1 d = depart1(c[k + 2], flag);
    const float ea = e[k + 1], eb = d.ob < 0 ? e[k] : e[k + 2];
    const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
    out[k] = fmaf(0.5f, fmaf(w, eb - ea, ea), p1[k + 2]);
  }
}

template <bool EVEN>
__global__ __launch_bounds__(kThreads, SLA_CEC3D_MIN_WAVES) void k_cec3d_seg(
    const float* __restrict__ phi, const float* __restrict__ ux, const float* __restrict__ uy,
    const float* __restrict__ uz, float* __restrict__ out, Geo g, int ychunk, int* flag) {
  using S = SegShape<EVEN>;
  constexpr int H = S::H, TA = S::TA, SA = S::SA, SB = S::SB, V = S::V;
  constexpr int KP = S::KP, KY = S::KY;
  __shared__ float P[S::NP];   // phi at the loaded plane, padded
  __shared__ float CA[S::NP];  // Courant numbers of the first sweep
  __shared__ float CB[S::NP];  // Courant numbers of the last sweep (output plane)
  __shared__ float AO[S::NP];  // first-sweep output (y-pipeline input)
  __shared__ float YO[S::NP];  // y-sweep output (last-sweep input)

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * S::TX, z0 = blockIdx.y * S::TZ;
  const int y0 = blockIdx.z * ychunk;
  const int y1 = min(y0 + ychunk, g.ny);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned nxy = unsigned(nx) * unsigned(ny);
  const float* uA = EVEN ? ux : uz;
  const float* uB = EVEN ? uz : ux;
  const float lamA = EVEN ? g.lam[0] : g.lam[2];
  const float lamB = EVEN ? g.lam[2] : g.lam[0];
  const float lamY = g.lam[1];

  unsigned poff[KP];
  unsigned yoff[KY];
  int ycol[KY];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int e = min(tid + k * kThreads, S::NP - 1);
    const int z = e / S::W - H, x = e % S::W - H;
    poff[k] = unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz));
  }
#pragma unroll
  for (int j = 0; j < KY; ++j) {
    const int e = min(tid + j * kThreads, S::NY - 1);
    const int z = S::YZ0 + e / S::YW, x = S::YX0 + e % S::YW;
    yoff[j] = unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz));
    ycol[j] = lidx<EVEN>(x, z);
  }
  auto pvalid = [&](int k) { return KP * kThreads == S::NP || tid + k * kThreads < S::NP; };
  auto yvalid = [&](int j) { return KY * kThreads == S::NY || tid + j * kThreads < S::NY; };

  // segment items: first sweep (line b, start a0), last sweep (line a, start b0)
  const bool has1 = tid < S::N1, has2 = tid < S::N2;
  const int i1 = EVEN ? lidx<EVEN>((tid % S::NS1) * V, tid / S::NS1 - H)
                      : lidx<EVEN>(tid / S::NS1 - H, (tid % S::NS1) * V);
  const int la2 = EVEN ? tid % TA : tid / S::NS2;  // last sweep: line (A coordinate)
  const int sb2 = EVEN ? tid / TA : tid % S::NS2;  // last sweep: segment index along B
  const int i2 = EVEN ? lidx<EVEN>(la2, sb2 * V) : lidx<EVEN>(sb2 * V, la2);
  const int ox2 = EVEN ? la2 : sb2 * V, oz2 = EVEN ? sb2 * V : la2;  // tile coords of out[0]

  float ra[3][KY], r1[3][KY], re[3][KY], rc[3][KY];
#pragma unroll
  for (int j = 0; j < KY; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  float fp[KP], fa[KP], fy[KY], fb[KY];
  auto prefetch = [&](int t) {
    const unsigned qoff = unsigned(wrap1(y0 - H + t, ny)) * unsigned(nx);
    const unsigned coff = unsigned(wrap1(y0 - H + t - 1, ny)) * unsigned(nx);
    const unsigned ooff = unsigned(wrap1(y0 + t - 2 * H, ny)) * unsigned(nx);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      fp[k] = phi[poff[k] + qoff];
      fa[k] = uA[poff[k] + qoff];
    }
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      fy[j] = uy[yoff[j] + coff];
      fb[j] = uB[yoff[j] + ooff];
    }
  };

  const int iters = (y1 - y0) + 2 * H;
  prefetch(0);
  auto body = [&](auto phase, int t) {
    constexpr int p0 = decltype(phase)::value;  // t % 3
    constexpr int p1 = (p0 + 2) % 3;            // (t - 1) % 3
    constexpr int p2 = (p0 + 1) % 3;            // (t - 2) % 3
    constexpr int p3 = p0;                      // (t - 3) % 3
    const bool emit = t >= 2 * H;

    // 1. publish the prefetched plane, then start fetching the next one
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (!pvalid(k)) continue;
      P[tid + k * kThreads] = fp[k];
      CA[tid + k * kThreads] = fa[k] * lamA;
    }
    float cy[KY];
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      cy[j] = fy[j] * lamY;
      if (emit && yvalid(j)) CB[ycol[j]] = fb[j] * lamB;
    }
    if (t + 1 < iters) prefetch(t + 1);
    __syncthreads();
    // 2. first sweep, one segment per thread
    if (has1) {
      float p[V + 6], c[V + 4], o[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) p[k] = P[i1 + (k - 3) * SA];
#pragma unroll
      for (int k = 0; k < V + 4; ++k) c[k] = CA[i1 + (k - 2) * SA];
      sweep_segment<V>(p, c, o, flag);
#pragma unroll
      for (int k = 0; k < V; ++k) AO[i1 + k * SA] = o[k];
    }
    __syncthreads();
    // 3. y sweep as a pipeline along the march (registers)
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      if (!yvalid(j)) continue;
      const int i = ycol[j];
      ra[p0][j] = AO[i];
      rc[p1][j] = cy[j];
      Dep1 d = depart1(rc[p1][j], flag);
      r1[p1][j] = lerp(ra[p1][j], d.ob < 0 ? ra[p2][j] : ra[p0][j], d.f);
      d = depart1(rc[p2][j], flag);
      re[p2][j] = ra[p2][j] - lerp(r1[p2][j], d.obr > 0 ? r1[p1][j] : r1[p3][j], d.f);
      d = depart1(rc[p3][j], flag);
      const float ea = re[p3][j];
      const float eb = d.ob < 0 ? re[p1][j] : re[p2][j];
      const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
      YO[i] = fmaf(0.5f, fmaf(w, eb - ea, ea), r1[p3][j]);
    }
    __syncthreads();
    if (!emit) return;
    // 4. last sweep, one segment per thread, stored to HBM at plane t - 6
    if (has2) {
      float p[V + 6], c[V + 4], o[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) p[k] = YO[i2 + (k - 3) * SB];
#pragma unroll
      for (int k = 0; k < V + 4; ++k) c[k] = CB[i2 + (k - 2) * SB];
      sweep_segment<V>(p, c, o, flag);
      const unsigned yo = unsigned(y0 + t - 2 * H) * unsigned(nx);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int x = x0 + ox2 + (EVEN ? 0 : k), z = z0 + oz2 + (EVEN ? k : 0);
        if (x < nx && z < nz) out[unsigned(x) + yo + nxy * unsigned(z)] = o[k];
      }
    }
    // the next plane stores CB before its first barrier
    __syncthreads();
  };

  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
}

}  // namespace

hipError_t launch_cec3d_seg(bool even, const Geo& g, const float* phi, const float* u, float* out,
                            int* flag, hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  const int ychunk = g.ny >= 256 ? 128 : 64;
  dim3 grid((g.nx + 63) / 64, (g.nz + 15) / 16, (g.ny + ychunk - 1) / ychunk);
  if (even)
    hipLaunchKernelGGL(k_cec3d_seg<true>, grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, ychunk, flag);
  else
    hipLaunchKernelGGL(k_cec3d_seg<false>, grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, ychunk, flag);
  return hipGetLastError();
}

hipError_t launch_cec3d(int R, bool even, const Geo& g, const float* phi, const float* u,
                        float* out, int* flag, hipStream_t st) {
  if (R != 1) return hipErrorInvalidValue;
  const size_t n = (size_t)g.ncells;
  const float* ux = u;
  const float* uy = u + n;
  const float* uz = u + 2 * n;
  const int ychunk = g.ny >= 256 ? 128 : 64;
  dim3 grid((g.nx + 63) / 64, (g.nz + 15) / 16, (g.ny + ychunk - 1) / ychunk);
  if (even)
    hipLaunchKernelGGL(k_cec3d_r1<true>, grid, dim3(kThreads), 0, st, phi, ux, uy, uz, out, g,
                       ychunk, flag);
  else
    hipLaunchKernelGGL(k_cec3d_r1<false>, grid, dim3(kThreads), 0, st, phi, ux, uy, uz, out, g,
                       ychunk, flag);
  return hipGetLastError();
}

}  // namespace sla
