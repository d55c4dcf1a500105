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

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace sla {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

// Reach-1 departure of a node with Courant number c (|c| < 1): fraction
// f = |c|; the far node of L_U is i - 1 if c >= 0 else i + 1 (ob < 0), the
// far node of L_{-U} is i + 1 if c > 0 else i - 1 (obr > 0).  A Courant
// number of magnitude 1 or more is detected once, where it is published to
// LDS (see `over`); the kernel then still reads only the nodes i-1..i+1.
struct Dep1 {
  float f;
  bool ob_neg;   // far node of L_U is i - 1
  bool obr_pos;  // far node of L_{-U} is i + 1
  int ob() const { return ob_neg ? -1 : 1; }
  int obr() const { return obr_pos ? 1 : -1; }
};

__device__ __forceinline__ Dep1 depart1(float c, int*) {
  Dep1 d;
  d.f = fabsf(c);
  d.ob_neg = c >= 0.f;
  d.obr_pos = c > 0.f;
  return d;
}

// True if |c| is beyond reach 1 (NaN is not an overflow: it propagates).
__device__ __forceinline__ bool over1(float c) { return fabsf(c) >= 1.f; }

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
// wrap any coordinate into [0, n)
__device__ __forceinline__ int wrapk(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Tile (x tile, z tile, y chunk) of this workgroup.  Workgroups are handed
// to the 8 XCDs round robin in launch order; with swz set, XCD k takes a
// contiguous range of the tile space instead (x fastest, then z, then the y
// chunk), so the tiles whose halos overlap run on the same XCD and share
// its L2.
__device__ __forceinline__ int3 block_tile(int swz) {
  if (!swz) return make_int3(blockIdx.x, blockIdx.y, blockIdx.z);
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned n = gx * gy * gridDim.z;
  const unsigned L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned xcd = L % 8u, q = n / 8u, r = n % 8u;
  const unsigned lg = xcd * q + min(xcd, r) + L / 8u;
  return make_int3(int(lg % gx), int((lg / gx) % gy), int(lg / (gx * gy)));
}

// Buffer accesses relative to a plane's start: the base lives in a scalar
// buffer descriptor built once per plane and each access is a 32-bit byte
// offset, so loads and stores need no per-access address arithmetic.
// Offsets stay below 2^32 because fused-step grids hold at most 2^30
// cells; the descriptor's size is the rest of the field (accesses beyond it
// read zero and write nothing).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
__device__ __forceinline__ Rsrc plane_rsrc(const float* base, size_t elems_left) {
  const unsigned bytes = elems_left >= (size_t(1) << 30) ? 0xFFFFFFFFu : unsigned(elems_left) * 4u;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), short(0), int(bytes), kRsrcWord3);
}
__device__ __forceinline__ float ld_at(Rsrc r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}
__device__ __forceinline__ void st_at(Rsrc r, unsigned byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 0);
}
// Access at a per-lane byte offset voff from the row or plane that starts
// soff bytes into the field (soff the same for the whole wave).  The
// descriptor is rebased on that row or plane (two scalar adds) and has the
// largest size a descriptor holds, so voff alone is range-checked.  A
// descriptor on the field's start cannot cover a field of 2^30 cells: its
// size tops out one byte short of 2^32, which would clip the last element.
// Callers keep voff + 4 <= 2^32 - 1: plane offsets go in soff whenever a
// plane is the march unit, and a row offset otherwise (then voff spans at
// most the field minus one row of planes: fine when ny >= 2 or the field
// holds fewer than 2^30 cells; the launchers check that).
__device__ __forceinline__ Rsrc based_rsrc(const float* field, unsigned soff) {
  // readfirstlane returns a signed int: widen the byte offset as unsigned
  const size_t off = unsigned(__builtin_amdgcn_readfirstlane(int(soff)));
  const char* b = reinterpret_cast<const char*>(field) + off;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), short(0), int(0xFFFFFFFFu), kRsrcWord3);
}
__device__ __forceinline__ float ld_vs(const float* field, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(based_rsrc(field, soff), voff, 0, 0));
}
__device__ __forceinline__ void st_vs(float* field, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), based_rsrc(field, soff), voff,
                                        0, 0);
}

// Prefetches are unconditional: a load under a condition merges the old and
// new register values, and the compiler then makes the wave wait for the
// loads it has just issued; past the end of a march they read valid
// (wrapped or repeated) planes whose values go unused.

// Minimum waves per SIMD the compiler must leave room for (register budget).
#ifndef SLA_CEC3D_MIN_WAVES
#define SLA_CEC3D_MIN_WAVES 2
#endif
#ifndef SLA_SEG_MIN_WAVES
#define SLA_SEG_MIN_WAVES 2
#endif

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
// A select between two elements of one register array is folded by the
// compiler into a dynamic index over the whole array (a compare chain); so
// every select below picks between two different arrays, the left and
// right neighbour views of the same values.
template <int V>
__device__ __forceinline__ void sweep_segment(const float (&p)[V + 6], const float (&c)[V + 4],
                                              float (&out)[V], int* flag) {
  float pl[V + 4], pr[V + 4];  // left / right neighbours of node a0-2+k
#pragma unroll
  for (int k = 0; k < V + 4; ++k) {
    pl[k] = p[k];
    pr[k] = p[k + 2];
  }
  float p1[V + 4];
#pragma unroll
  for (int k = 0; k < V + 4; ++k) {  // node a0-2+k
    const Dep1 d = depart1(c[k], flag);
    p1[k] = lerp(p[k + 1], d.ob_neg ? pl[k] : pr[k], d.f);
  }
  float ql[V + 2], qr[V + 2];  // neighbours of Phi1 at node a0-1+k
#pragma unroll
  for (int k = 0; k < V + 2; ++k) {
    ql[k] = p1[k];
    qr[k] = p1[k + 2];
  }
  float e[V + 2];
#pragma unroll
  for (int k = 0; k < V + 2; ++k) {  // node a0-1+k
    const Dep1 d = depart1(c[k + 1], flag);
    e[k] = p[k + 2] - lerp(p1[k + 1], d.obr_pos ? qr[k] : ql[k], d.f);
  }
  float el[V], er[V];  // neighbours of e at node a0+k
#pragma unroll
  for (int k = 0; k < V; ++k) {
    el[k] = e[k];
    er[k] = e[k + 2];
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {  // node a0+k
    const Dep1 d = depart1(c[k + 2], flag);
    const float ea = e[k + 1], eb = d.ob_neg ? el[k] : er[k];
    const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
    out[k] = fmaf(0.5f, fmaf(w, eb - ea, ea), p1[k + 2]);
  }
}

template <bool EVEN>
__global__ __launch_bounds__(kThreads, SLA_SEG_MIN_WAVES) void k_cec3d_seg(
    const float* __restrict__ phi, const float* __restrict__ ux, const float* __restrict__ uy,
    const float* __restrict__ uz, float* __restrict__ out, Geo g, int ychunk, int swz, int* flag) {
  using S = SegShape<EVEN>;
  constexpr int H = S::H, TA = S::TA, SA = S::SA, SB = S::SB, V = S::V;
  constexpr int KP = S::KP, KY = S::KY;
  __shared__ float P[S::NP];   // phi at the loaded plane, padded
  __shared__ float CA[S::NP];  // Courant numbers of the first sweep
  __shared__ float CB[S::NP];  // Courant numbers of the last sweep (output plane)
  __shared__ float AO[S::NP];  // first-sweep output (y-pipeline input)
  __shared__ float YO[S::NP];  // y-sweep output (last-sweep input)

  const int tid = threadIdx.x;
  const int3 bt = block_tile(swz);
  const int x0 = bt.x * S::TX, z0 = bt.y * S::TZ;
  const int y0 = bt.z * ychunk;
  const int y1 = min(y0 + ychunk, g.ny);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned nxy = unsigned(nx) * unsigned(ny);
  const float* uA = EVEN ? ux : uz;
  const float* uB = EVEN ? uz : ux;
  const float lamA = EVEN ? g.lam[0] : g.lam[2];
  const float lamB = EVEN ? g.lam[2] : g.lam[0];
  const float lamY = g.lam[1];

  // byte offsets (x-z part) of this thread's cells within a y plane
  unsigned poff[KP];
  unsigned yoff[KY];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int e = min(tid + k * kThreads, S::NP - 1);
    const int z = e / S::W - H, x = e % S::W - H;
    poff[k] = 4u * (unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz)));
  }
#pragma unroll
  for (int j = 0; j < KY; ++j) {
    const int e = min(tid + j * kThreads, S::NY - 1);
    const int z = S::YZ0 + e / S::YW, x = S::YX0 + e % S::YW;
    yoff[j] = 4u * (unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz)));
  }
  // LDS index of y column j (region element tid + 256 j): the region is
  // 64-wide rows (even) or whole padded rows (odd), so consecutive j are a
  // fixed stride apart and only the first index is kept in a register
  static_assert(EVEN ? (kThreads % S::YW == 0) : (S::YW == S::W), "y columns a fixed stride apart");
  const int ycol0 = lidx<EVEN>(S::YX0 + tid % S::YW, S::YZ0 + tid / S::YW);
  constexpr int YCS = EVEN ? (kThreads / S::YW) * S::W : kThreads;
  auto ycol = [&](int j) { return ycol0 + j * YCS; };
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
  // byte offset of out[0] within a y plane, the step between outputs, and
  // how many of the V outputs are inside the grid
  const unsigned ostep2 = EVEN ? 4u * nxy : 4u;
  const unsigned obase2 = 4u * (unsigned(min(x0 + ox2, nx - 1)) + nxy * unsigned(min(z0 + oz2, nz - 1)));
  const int nvalid2 = EVEN ? (x0 + ox2 < nx ? min(V, nz - (z0 + oz2)) : 0)
                           : (z0 + oz2 < nz ? min(V, nx - (x0 + ox2)) : 0);

  float ra[3][KY], r1[3][KY], re[3][KY], rc[3][KY];
#pragma unroll
  for (int j = 0; j < KY; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  float fp[KP], fa[KP], fy[KY], fb[KY];
  auto prefetch = [&](int t) {
    const size_t qoff = size_t(wrap1(y0 - H + t, ny)) * size_t(nx);
    const size_t coff = size_t(wrap1(y0 - H + t - 1, ny)) * size_t(nx);
    const size_t ooff = size_t(wrap1(y0 + t - 2 * H, ny)) * size_t(nx);
    const size_t ncells = size_t(nxy) * size_t(nz);
    const Rsrc pq = plane_rsrc(phi + qoff, ncells - qoff);
    const Rsrc aq = plane_rsrc(uA + qoff, ncells - qoff);
    const Rsrc yq = plane_rsrc(uy + coff, ncells - coff);
    const Rsrc bq = plane_rsrc(uB + ooff, ncells - ooff);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      fp[k] = ld_at(pq, poff[k]);
      fa[k] = ld_at(aq, poff[k]);
    }
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      fy[j] = ld_at(yq, yoff[j]);
      fb[j] = ld_at(bq, yoff[j]);
    }
  };

  const int iters = (y1 - y0) + 2 * H;
  bool over = false;  // a Courant number beyond reach 1 was published
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
      const float ca = fa[k] * lamA;
      over |= over1(ca);
      P[tid + k * kThreads] = fp[k];
      CA[tid + k * kThreads] = ca;
    }
    float cy[KY];
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      cy[j] = fy[j] * lamY;
      over |= over1(cy[j]);
      if (emit && yvalid(j)) {
        const float cb = fb[j] * lamB;
        over |= over1(cb);
        CB[ycol(j)] = cb;
      }
    }
    prefetch(min(t + 1, iters - 1));  // unconditional (see the top of the file)
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
      const int i = ycol(j);
      ra[p0][j] = AO[i];
      rc[p1][j] = cy[j];
      Dep1 d = depart1(rc[p1][j], flag);
      r1[p1][j] = lerp(ra[p1][j], d.ob_neg ? ra[p2][j] : ra[p0][j], d.f);
      d = depart1(rc[p2][j], flag);
      re[p2][j] = ra[p2][j] - lerp(r1[p2][j], d.obr_pos ? r1[p1][j] : r1[p3][j], d.f);
      d = depart1(rc[p3][j], flag);
      const float ea = re[p3][j];
      const float eb = d.ob_neg ? re[p1][j] : re[p2][j];
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
      const size_t orow = size_t(y0 + t - 2 * H) * size_t(nx);
      const Rsrc oq = plane_rsrc(out + orow, size_t(nxy) * size_t(nz) - orow);
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (k < nvalid2) st_at(oq, obase2 + k * ostep2, o[k]);
    }
    // the next plane stores CB before its first barrier
    __syncthreads();
  };

  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

// ---------------------------------------------------------------------------
// Window-march variants (4: V = 4, 6: V = 8): no LDS and no barriers; every
// wave works alone.
// A wave covers a window of 64 consecutive x (one node per lane, the 58
// middle lanes produce outputs) and a segment of V rows of a second axis,
// and marches along the third.  The sweep along x reads the neighbour
// values from the adjacent lanes; the sweep along the segment axis runs
// in each thread's registers (sweep_segment, the segment grown by the 3-row
// halo); the sweep along the march axis is the register pipeline.
//   even step (x, y, z): x across lanes, y in the segment, z along the march;
//   odd step  (z, y, x): z in the segment, y along the march, x across lanes.
// Loads and stores use a per-lane byte offset (x) plus a row/plane offset
// that is the same for the whole wave (scalar registers).  Each segment
// reads V + 6 rows of phi for V rows of output, so longer segments read
// less (V = 8: 1.45x the algorithmic loads issued against 1.79x for V = 4)
// but hold twice the registers.
// ---------------------------------------------------------------------------
constexpr int kWmUse = 58;  // outputs per 64-lane window (reach 1: 3 halo lanes a side)

// Wrapped indices of five consecutive march planes, advanced by one plane at
// a time without a division (the values are the same for the whole wave).
struct PlaneWin {
  int p[6];
  int n;
  __device__ PlaneWin(int first, int n_) : n(n_) {
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = __builtin_amdgcn_readfirstlane(wrapk(first + k, n));
  }
  __device__ void advance() {
#pragma unroll
    for (int k = 0; k < 5; ++k) p[k] = p[k + 1];
    p[5] = p[5] + 1 < n ? p[5] + 1 : 0;
  }
  __device__ int plane(int k) const { return p[k]; }
};

// Store V output rows of one plane: rows j < rows_left only (a uniform
// test per row), lanes with lane_out only (one exec-mask region).
// roff: per-lane byte offsets of the rows within a plane; q: the plane's.
template <int V>
__device__ __forceinline__ void store_rows(float* ro, const unsigned* roff, unsigned q,
                                           const float (&o)[V], bool lane_out, int rows_left) {
  if (!lane_out) return;
  if (rows_left >= V) {
#pragma unroll
    for (int j = 0; j < V; ++j) st_vs(ro, roff[j], q, o[j]);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (j < rows_left) st_vs(ro, roff[j], q, o[j]);
  }
}

// Value of the lane below (lane - 1) and above (lane + 1): DPP wave shifts
// (one vector move each, which the compiler can fold into the instruction
// that uses it); lanes 0 and 63 receive 0.  Only halo lanes see those
// zeros: a sweep's output is valid three lanes in from the window's edges.
__device__ __forceinline__ float from_below(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, i, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_above(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, i, 0x130, 0xf, 0xf, true));
}

// Third-order sweep along x of one node per lane (lanes are consecutive x);
// the values of lanes 0 and 63 are not valid (their neighbours are outside).
__device__ __forceinline__ float xsweep_lanes(float p, float c) {
  const Dep1 d = depart1(c, nullptr);
  const float pm = from_below(p), pp = from_above(p);
  const float p1 = lerp(p, d.ob_neg ? pm : pp, d.f);
  const float qm = from_below(p1), qp = from_above(p1);
  const float e = p - lerp(p1, d.obr_pos ? qp : qm, d.f);
  const float em = from_below(e), ep = from_above(e);
  const float eb = d.ob_neg ? em : ep;
  const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
  return fmaf(0.5f, fmaf(w, eb - e, e), p1);
}

// One step of the register pipeline along the march for V columns: a (the
// new plane's input) enters at ring slot p0, cprev is the Courant number of
// the previous plane; returns in out the output of the plane three back.
template <int V, int P0>
__device__ __forceinline__ void march_step(float (&ra)[3][V], float (&r1)[3][V], float (&re)[3][V],
                                           float (&rc)[3][V], const float (&a)[V],
                                           const float (&cprev)[V], float (&out)[V]) {
  constexpr int p0 = P0, p1 = (P0 + 2) % 3, p2 = (P0 + 1) % 3, p3 = P0;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    ra[p0][j] = a[j];
    rc[p1][j] = cprev[j];
    Dep1 d = depart1(rc[p1][j], nullptr);
    r1[p1][j] = lerp(ra[p1][j], d.ob_neg ? ra[p2][j] : ra[p0][j], d.f);
    d = depart1(rc[p2][j], nullptr);
    re[p2][j] = ra[p2][j] - lerp(r1[p2][j], d.obr_pos ? r1[p1][j] : r1[p3][j], d.f);
    d = depart1(rc[p3][j], nullptr);
    const float ea = re[p3][j];
    const float eb = d.ob_neg ? re[p1][j] : re[p2][j];
    const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
    out[j] = fmaf(0.5f, fmaf(w, eb - ea, ea), r1[p3][j]);
  }
}

template <bool EVEN, int V>
__global__ __launch_bounds__(kThreads) void k_cec3d_wm(const float* __restrict__ phi,
                                                       const float* __restrict__ ux,
                                                       const float* __restrict__ uy,
                                                       const float* __restrict__ uz,
                                                       float* __restrict__ out, Geo g, int chunk,
                                                       int swz, int* flag) {
  const int lane = threadIdx.x & 63;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  // segment axis: y (even) or z (odd); march axis: z (even) or y (odd)
  const int ns = EVEN ? ny : nz, nm = EVEN ? nz : ny;
  const int nwx = (nx + kWmUse - 1) / kWmUse, nseg = (ns + V - 1) / V;
  const int nch = (nm + chunk - 1) / chunk;
  const int3 bt = block_tile(swz);  // 1D grid: bt.x is the (XCD-mapped) block
  const int wid = bt.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (wid >= nwx * nseg * nch) return;  // the whole wave
  const int wx = wid % nwx, sg = (wid / nwx) % nseg, ch = wid / (nwx * nseg);
  const int xw = wx * kWmUse - 3 + lane;  // this lane's x (before wrap)
  const unsigned vx = 4u * unsigned(wrapk(xw, nx));
  const unsigned rowb = 4u * unsigned(nx), plb = 4u * unsigned(nx) * unsigned(ny);
  const unsigned sstr = EVEN ? rowb : plb;  // bytes per segment-axis step
  const unsigned mstr = EVEN ? plb : rowb;  // bytes per march-axis step
  const int s0 = sg * V, m0 = ch * chunk, m1 = min(m0 + chunk, nm);
  // per-lane byte offsets of the segment rows s0 - 3 .. s0 + V + 2 within a
  // march plane (the plane's offset goes in the instructions' scalar part)
  unsigned vrow[V + 6];
#pragma unroll
  for (int k = 0; k < V + 6; ++k)
    vrow[k] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(s0 - 3 + k, ns))) * sstr;
  const float *rp = phi, *rx = ux;
  float* ro = out;
  // first sweep's velocity (along x if even, along the segment if odd)
  const float* rA = EVEN ? ux : uz;
  const float* rS = EVEN ? uy : uz;  // segment-axis velocity
  const float* rM = EVEN ? uz : uy;  // march-axis velocity
  const float lamX = g.lam[0], lamS = EVEN ? g.lam[1] : g.lam[2], lamM = EVEN ? g.lam[2] : g.lam[1];
  // wrapped march-plane indices of planes m0 - 6 + t .. m0 - 2 + t at
  // iteration t, advanced by one plane per iteration (uniform, scalar)
  PlaneWin pw(m0 - 6, nm);

  // prefetched inputs of iteration t (march plane q_t = m0 - 3 + t)
  float fp[V + 6];  // phi on the segment rows (+halo)
  float fa[V + 6];  // even: x velocity on the same rows; odd: unused
  float fs[V + 4];  // segment-axis velocity on rows s0 - 2 .. s0 + V + 1
  float fm[V];      // march-axis velocity of plane q_{t-1}, rows s0 .. s0 + V - 1
  float fx[V];      // odd: x velocity of the output plane q_{t-3}
  // planes q_t, q_{t-1}, q_{t-3} of the iteration being prefetched (ahead =
  // 0 for iteration t, 1 for t + 1)
  auto prefetch = [&](int ahead) {
    const unsigned q = unsigned(pw.p[3 + ahead]) * mstr, qm1 = unsigned(pw.p[2 + ahead]) * mstr,
                   qo = unsigned(pw.p[ahead]) * mstr;
#pragma unroll
    for (int k = 0; k < V + 6; ++k) {
      fp[k] = ld_vs(rp, vrow[k], q);
      if (EVEN) fa[k] = ld_vs(rA, vrow[k], q);
    }
#pragma unroll
    for (int k = 0; k < V + 4; ++k) fs[k] = ld_vs(rS, vrow[k + 1], q);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      fm[j] = ld_vs(rM, vrow[j + 3], qm1);
      if (!EVEN) fx[j] = ld_vs(rx, vrow[j + 3], qo);
    }
  };

  float ra[3][V], r1[3][V], re[3][V], rc[3][V];
#pragma unroll
  for (int j = 0; j < V; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  const int iters = (m1 - m0) + 6;
  const bool lane_out = lane >= 3 && lane < 61 && wx * kWmUse + lane - 3 < nx;
  bool over = false;
  prefetch(0);
  auto body = [&](auto phase, int t) {
    constexpr int P0 = decltype(phase)::value;
    float p[V + 6], cs[V + 4], cm[V], a[V], o[V];
    float cxo[V];
#pragma unroll
    for (int k = 0; k < V + 6; ++k) {
      p[k] = fp[k];
      if (EVEN) {
        const float c = fa[k] * lamX;
        over |= over1(c);
        p[k] = xsweep_lanes(p[k], c);  // first sweep (x) of this row
      }
    }
#pragma unroll
    for (int k = 0; k < V + 4; ++k) {
      cs[k] = fs[k] * lamS;
      over |= over1(cs[k]);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      cm[j] = fm[j] * lamM;
      over |= over1(cm[j]);
      cxo[j] = EVEN ? 0.f : fx[j] * lamX;
      if (!EVEN) over |= over1(cxo[j]);
    }
    prefetch(1);  // unconditional (see the top of the file)
    // sweep along the segment axis (second for even, first for odd)
    sweep_segment<V>(p, cs, a, flag);
    // sweep along the march axis (even: last; odd: second)
    march_step<V, P0>(ra, r1, re, rc, a, cm, o);
    if (t >= 6) {
      const unsigned qo = unsigned(pw.p[0]) * mstr;
      if (!EVEN)
#pragma unroll
        for (int j = 0; j < V; ++j) o[j] = xsweep_lanes(o[j], cxo[j]);  // last sweep (x)
      store_rows<V>(ro, vrow + 3, qo, o, lane_out, ns - s0);
    }
    pw.advance();
  };
  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

// Window-march launch geometry: waves per march layer and the wave count
// for a march chunk of c planes.
struct WmShape {
  long long layer;  // x windows x segments
  int nm;           // march-axis length
  long long waves(int c) const { return layer * ((nm + c - 1) / c); }
};
WmShape wm_shape(bool even, const Geo& g, int V) {
  const int ns = even ? g.ny : g.nz, nm = even ? g.nz : g.ny;
  return {(long long)((g.nx + kWmUse - 1) / kWmUse) * ((ns + V - 1) / V), nm};
}
// With 8-row segments a wave needs about 200 registers: 2 waves per SIMD,
// 2048 on the chip (256 CUs).  Such long waves run best when the launch is
// one nearly full pass over the chip or at least four (the last partial
// pass then costs little).
constexpr long long kWm8Resident = 2048;
bool wm8_fills(long long waves) {
  return (waves >= kWm8Resident * 9 / 10 && waves <= kWm8Resident) || waves >= 4 * kWm8Resident;
}
// March chunk (planes per wave), measured best at 256^3 .. 1024^3:
// 4-row segments take 64 unless that leaves fewer than 3840 waves (15 per
// CU), then 32, then 16; 8-row segments take the largest of 64, 32 that
// fills the chip (above), else 16.
int wm_default_chunk(const WmShape& s, int V) {
  for (int c : {64, 32})
    if (V >= 8 ? wm8_fills(s.waves(c)) : s.waves(c) >= 3840) return c;
  return 16;
}

template <int V>
hipError_t launch_cec3d_wm(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc) {
  const size_t n = (size_t)g.ncells;
  const WmShape s = wm_shape(even, g, V);
  const int chunk = lc.ychunk > 0 ? lc.ychunk : wm_default_chunk(s, V);
  dim3 grid(unsigned((s.waves(chunk) + 3) / 4));
  if (even)
    hipLaunchKernelGGL((k_cec3d_wm<true, V>), grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, chunk, lc.swizzle, flag);
  else
    hipLaunchKernelGGL((k_cec3d_wm<false, V>), grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, chunk, lc.swizzle, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Window march with shared segment halos (variant 7).  A workgroup of WX x W
// waves takes WX consecutive 64-lane x windows and, in each, W consecutive
// V-row segments (S = W*V rows), and marches them together along the third
// axis.  The S + 6 rows the segment-axis sweep reads are loaded once per
// window instead of V + 6 per wave: wave w of a window loads the
// R = V + 6/W rows w*R .. w*R + R - 1 of the grown segment, stores what the
// segment sweep needs in LDS (even: the x-swept phi and the y Courant
// numbers; odd: phi and the z Courant numbers), and after one barrier per
// march plane every wave reads its V + 6 rows back.  The neighbouring
// windows of one workgroup share the 128-byte lines their 3-lane x halos
// straddle.  The LDS is double-buffered, so a wave writing plane t+1 never
// meets one still reading plane t.  The march-axis velocity (and on odd
// steps the x velocity of the output plane) is read for the wave's own
// rows only.  Windows past the row's end (when WX does not divide the
// window count) only take part in the barriers.  Same FP32 operations per
// node as the other variants.
// ---------------------------------------------------------------------------
template <bool EVEN, int V, int W, int WX>
__global__ __launch_bounds__(64 * W * WX) void k_cec3d_wl(const float* __restrict__ phi,
                                                          const float* __restrict__ ux,
                                                          const float* __restrict__ uy,
                                                          const float* __restrict__ uz,
                                                          float* __restrict__ out, Geo g, int chunk,
                                                          int swz, int* flag) {
  static_assert(6 % W == 0, "the 6 halo rows must split evenly over the waves");
  constexpr int S = V * W, R = V + 6 / W, NR = S + 6;
  __shared__ float lp[2][WX][NR][64];  // segment sweep input (phi, x-swept if even)
  __shared__ float lc[2][WX][NR][64];  // segment-axis Courant numbers
  const int lane = threadIdx.x & 63, xi = (threadIdx.x >> 6) % WX, w = (threadIdx.x >> 6) / WX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ns = EVEN ? ny : nz, nm = EVEN ? nz : ny;
  const int nwx = (nx + kWmUse - 1) / kWmUse, ngx = (nwx + WX - 1) / WX, ngs = (ns + S - 1) / S;
  const int nch = (nm + chunk - 1) / chunk;
  const int blk = block_tile(swz).x;  // 1D grid, XCD-mapped
  if (blk >= ngx * ngs * nch) return;  // the whole workgroup
  const int wx0 = (blk % ngx) * WX, gs = (blk / ngx) % ngs, ch = blk / (ngx * ngs);
  const bool wx_ok = wx0 + xi < nwx;  // the same for the whole wave
  const int wx = min(wx0 + xi, nwx - 1);
  const int xw = wx * kWmUse - 3 + lane;
  const unsigned vx = 4u * unsigned(wrapk(xw, nx));
  const unsigned rowb = 4u * unsigned(nx), plb = 4u * unsigned(nx) * unsigned(ny);
  const unsigned sstr = EVEN ? rowb : plb, mstr = EVEN ? plb : rowb;
  const int g0 = gs * S, s0 = g0 + w * V, m0 = ch * chunk, m1 = min(m0 + chunk, nm);
  // per-lane byte offsets within a march plane of the rows this wave loads
  // (grown-segment rows w*R + k) and of its output rows
  unsigned loff[R], ooff[V];
#pragma unroll
  for (int k = 0; k < R; ++k)
    loff[k] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(g0 - 3 + w * R + k, ns))) * sstr;
#pragma unroll
  for (int j = 0; j < V; ++j)
    ooff[j] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(s0 + j, ns))) * sstr;
  const float *rp = phi, *rx = ux;
  float* ro = out;
  const float* rS = EVEN ? uy : uz;  // segment-axis velocity
  const float* rM = EVEN ? uz : uy;  // march-axis velocity
  const float lamX = g.lam[0], lamS = EVEN ? g.lam[1] : g.lam[2], lamM = EVEN ? g.lam[2] : g.lam[1];
  PlaneWin pw(m0 - 6, nm);  // planes m0 - 6 + t .. m0 - 2 + t at iteration t

  float fp[R], fa[R], fs[R];  // phi, x velocity (even), segment velocity on the loaded rows
  float fm[V], fx[V];         // march velocity of plane q-1; odd: x velocity of the output plane
  auto prefetch = [&](int ahead) {  // 0: iteration t; 1: iteration t + 1
    const unsigned q = unsigned(pw.p[3 + ahead]) * mstr, qm1 = unsigned(pw.p[2 + ahead]) * mstr,
                   qo = unsigned(pw.p[ahead]) * mstr;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      fp[k] = ld_vs(rp, loff[k], q);
      if (EVEN) fa[k] = ld_vs(rx, loff[k], q);
      fs[k] = ld_vs(rS, loff[k], q);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      fm[j] = ld_vs(rM, ooff[j], qm1);
      if (!EVEN) fx[j] = ld_vs(rx, ooff[j], qo);
    }
  };

  float ra[3][V], r1[3][V], re[3][V], rc[3][V];
#pragma unroll
  for (int j = 0; j < V; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  const int iters = (m1 - m0) + 6;
  const bool lane_out = lane >= 3 && lane < 61 && wx * kWmUse + lane - 3 < nx;
  bool over = false;
  if (wx_ok) prefetch(0);
  auto body = [&](auto phase, int t) {
    constexpr int P0 = decltype(phase)::value;
    const int b = t & 1;
    if (!wx_ok) {  // a window past the row's end: barriers only
      __syncthreads();
      return;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      float v = fp[k];
      if (EVEN) {
        const float c = fa[k] * lamX;
        over |= over1(c);
        v = xsweep_lanes(v, c);  // first sweep (x) of this row
      }
      const float c = fs[k] * lamS;
      over |= over1(c);
      lp[b][xi][w * R + k][lane] = v;
      lc[b][xi][w * R + k][lane] = c;
    }
    float cm[V], cxo[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      cm[j] = fm[j] * lamM;
      over |= over1(cm[j]);
      cxo[j] = EVEN ? 0.f : fx[j] * lamX;
      if (!EVEN) over |= over1(cxo[j]);
    }
    prefetch(1);  // unconditional (see the top of the file)
    __syncthreads();
    float p[V + 6], cs[V + 4], a[V], o[V];
#pragma unroll
    for (int k = 0; k < V + 6; ++k) p[k] = lp[b][xi][w * V + k][lane];
#pragma unroll
    for (int k = 0; k < V + 4; ++k) cs[k] = lc[b][xi][w * V + 1 + k][lane];
    // sweep along the segment axis (second for even, first for odd)
    sweep_segment<V>(p, cs, a, flag);
    // sweep along the march axis (even: last; odd: second)
    march_step<V, P0>(ra, r1, re, rc, a, cm, o);
    if (t >= 6) {
      const unsigned qo = unsigned(pw.p[0]) * mstr;
      if (!EVEN)
#pragma unroll
        for (int j = 0; j < V; ++j) o[j] = xsweep_lanes(o[j], cxo[j]);  // last sweep (x)
      store_rows<V>(ro, ooff, qo, o, lane_out, ns - s0);
    }
    pw.advance();
  };
  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

// x windows per workgroup of the shared-halo march: 3 or 2 when that divides
// the window count (no surplus windows), else 0 (no such choice).
int wl_windows(const Geo& g) {
  const int nwx = (g.nx + kWmUse - 1) / kWmUse;
  return nwx % 3 == 0 ? 3 : nwx % 2 == 0 ? 2 : 0;
}

// V = 8 rows per wave, W = 2 waves per window, WX windows per workgroup
// (3 if that divides the window count, else 2).  March chunk: 64 planes
// unless that leaves fewer than 512 workgroups (two per CU), then 32, then 16.
template <int WX>
hipError_t launch_cec3d_wl_x(bool even, const Geo& g, const float* phi, const float* u, float* out,
                             int* flag, hipStream_t st, Cec3dLaunch lc) {
  constexpr int V = 8, W = 2;
  const size_t n = (size_t)g.ncells;
  const int ns = even ? g.ny : g.nz, nm = even ? g.nz : g.ny;
  const long long groups =
      (long long)(((g.nx + kWmUse - 1) / kWmUse + WX - 1) / WX) * ((ns + V * W - 1) / (V * W));
  int chunk = lc.ychunk;
  if (chunk <= 0) {
    chunk = 16;
    for (int c : {64, 32})
      if (groups * ((nm + c - 1) / c) >= 512) { chunk = c; break; }
  }
  dim3 grid(unsigned(groups * ((nm + chunk - 1) / chunk)));
  if (even)
    hipLaunchKernelGGL((k_cec3d_wl<true, V, W, WX>), grid, dim3(64 * W * WX), 0, st, phi, u, u + n,
                       u + 2 * n, out, g, chunk, lc.swizzle, flag);
  else
    hipLaunchKernelGGL((k_cec3d_wl<false, V, W, WX>), grid, dim3(64 * W * WX), 0, st, phi, u, u + n,
                       u + 2 * n, out, g, chunk, lc.swizzle, flag);
  return hipGetLastError();
}
hipError_t launch_cec3d_wl(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc) {
  return wl_windows(g) == 3 ? launch_cec3d_wl_x<3>(even, g, phi, u, out, flag, st, lc)
                            : launch_cec3d_wl_x<2>(even, g, phi, u, out, flag, st, lc);
}

// ---------------------------------------------------------------------------
// Persistent shared-halo window march (variant 8).  The work of the
// shared-halo march (a group of WX 64-lane x windows by S = V*W rows of the
// segment axis, marched along the third axis) is cut into runs: the groups
// are laid end to end, plane after plane, and workgroup b takes the range
// [b*span, (b+1)*span) of that line, so a launch of about one workgroup per
// CU leaves no tail and a workgroup restarts its march pipeline only where
// its range crosses into the next group (6 extra planes per restart, against
// one per march chunk in variant 7).  The S + 6 rows the segment sweep reads
// are split over the W waves of a window as evenly as possible.  Same FP32
// operations per node as the other variants.
// ---------------------------------------------------------------------------
template <bool EVEN, int V, int W, int WX, int PF>
__global__ __launch_bounds__(64 * W * WX) void k_cec3d_wp(const float* __restrict__ phi,
                                                          const float* __restrict__ ux,
                                                          const float* __restrict__ uy,
                                                          const float* __restrict__ uz,
                                                          float* __restrict__ out, Geo g, int span,
                                                          int* flag) {
  constexpr int S = V * W, NR = S + 6, RW = (NR + W - 1) / W;
  __shared__ float lp[2][WX][NR][64];  // segment sweep input (phi, x-swept if even)
  __shared__ float lc[2][WX][NR][64];  // segment-axis Courant numbers
  const int lane = threadIdx.x & 63, xi = (threadIdx.x >> 6) % WX, w = (threadIdx.x >> 6) / WX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ns = EVEN ? ny : nz, nm = EVEN ? nz : ny;
  const int nwx = (nx + kWmUse - 1) / kWmUse, ngx = (nwx + WX - 1) / WX, ngs = (ns + S - 1) / S;
  const long long total = (long long)ngx * ngs * nm;
  const int blk = block_tile(1).x;  // XCD-mapped 1D grid
  long long i0, i1;
  if (span > 0) {  // a range of the line of groups
    i0 = (long long)blk * span;
    i1 = min(i0 + (long long)span, total);
  } else {  // one chunk of -span planes of one group, groups fastest
    const int ng = ngx * ngs, ch = blk / ng, grp = blk - ch * ng;
    i0 = (long long)grp * nm + (long long)ch * -span;
    i1 = (long long)grp * nm + min(nm, (ch + 1) * -span);
  }
  const unsigned rowb = 4u * unsigned(nx), plb = 4u * unsigned(nx) * unsigned(ny);
  const unsigned sstr = EVEN ? rowb : plb, mstr = EVEN ? plb : rowb;
  const float* rS = EVEN ? uy : uz;  // segment-axis velocity
  const float* rM = EVEN ? uz : uy;  // march-axis velocity
  const float lamX = g.lam[0], lamS = EVEN ? g.lam[1] : g.lam[2], lamM = EVEN ? g.lam[2] : g.lam[1];
  // rows this wave loads: grown-segment rows w*RW + k (k < nld); every wave
  // loads its first kAll rows
  constexpr int kAll = NR - (W - 1) * RW;
  const int nld = min(RW, NR - w * RW);
  bool over = false;
  while (i0 < i1) {  // one run: the same for every wave of the workgroup
    const int grp = int(i0 / nm), m0 = int(i0 - (long long)grp * nm);
    const int m1 = int(min((long long)nm, (long long)m0 + (i1 - i0)));
    i0 += m1 - m0;
    const int wx0 = (grp % ngx) * WX, gs = grp / ngx;
    const bool wx_ok = wx0 + xi < nwx;  // the same for the whole wave
    const int wx = min(wx0 + xi, nwx - 1);
    const unsigned vx = 4u * unsigned(wrapk(wx * kWmUse - 3 + lane, nx));
    const int g0 = gs * S, s0 = g0 + w * V;
    // per-lane byte offsets within a march plane of the rows this wave loads
    // and of its output rows (the plane's offset goes in the scalar part)
    unsigned lrow[RW], orow[V];
#pragma unroll
    for (int k = 0; k < RW; ++k)
      lrow[k] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(g0 - 3 + w * RW + k, ns))) * sstr;
#pragma unroll
    for (int j = 0; j < V; ++j)
      orow[j] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(s0 + j, ns))) * sstr;
    PlaneWin pw(m0 - 6, nm);  // planes m0 - 6 + t .. m0 - 2 + t at iteration t

    // inputs of PF iterations ahead in flight: PF = 1, one set of registers
    // (consumed, then reloaded); PF = 2, three (one consumed, two loading),
    // the set of iteration t being t mod 3, the phase of the ring
    constexpr int NB = PF == 1 ? 1 : 3;
    float fp[NB][RW], fa[NB][RW], fs[NB][RW];  // phi, x velocity (even), segment velocity
    float fm[NB][V], fx[NB][V];  // march velocity of plane q-1; odd: x velocity of the output plane
    auto prefetch = [&](auto setc, int ahead) {  // ahead: iterations after the current one
      constexpr int B = decltype(setc)::value;
      const unsigned q = unsigned(pw.plane(3 + ahead)) * mstr,
                     qm1 = unsigned(pw.plane(2 + ahead)) * mstr, qo = unsigned(pw.plane(ahead)) * mstr;
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        if (k < kAll || k < nld) {
          fp[B][k] = ld_vs(phi, lrow[k], q);
          if (EVEN) fa[B][k] = ld_vs(ux, lrow[k], q);
          fs[B][k] = ld_vs(rS, lrow[k], q);
        }
      }
#pragma unroll
      for (int j = 0; j < V; ++j) {
        fm[B][j] = ld_vs(rM, orow[j], qm1);
        if (!EVEN) fx[B][j] = ld_vs(ux, orow[j], qo);
      }
    };

    float ra[3][V], r1[3][V], re[3][V], rc[3][V];
#pragma unroll
    for (int j = 0; j < V; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

    const int iters = (m1 - m0) + 6;
    const bool lane_out = lane >= 3 && lane < 61 && wx * kWmUse + lane - 3 < nx;
    if (wx_ok) {
      prefetch(std::integral_constant<int, 0>{}, 0);
      if (PF == 2) prefetch(std::integral_constant<int, NB == 1 ? 0 : 1>{}, 1);
    }
    auto body = [&](auto phase, int t) {
      constexpr int P0 = decltype(phase)::value;
      constexpr int B = NB == 1 ? 0 : P0;  // this iteration's inputs
      const int b = t & 1;
      if (!wx_ok) {  // a window past the row's end: barriers only
        __syncthreads();
        return;
      }
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        if (k < kAll || k < nld) {
          float v = fp[B][k];
          if (EVEN) {
            const float c = fa[B][k] * lamX;
            over |= over1(c);
            v = xsweep_lanes(v, c);  // first sweep (x) of this row
          }
          const float c = fs[B][k] * lamS;
          over |= over1(c);
          lp[b][xi][w * RW + k][lane] = v;
          lc[b][xi][w * RW + k][lane] = c;
        }
      }
      float cm[V], cxo[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        cm[j] = fm[B][j] * lamM;
        over |= over1(cm[j]);
        cxo[j] = EVEN ? 0.f : fx[B][j] * lamX;
        if (!EVEN) over |= over1(cxo[j]);
      }
      prefetch(std::integral_constant<int, NB == 1 ? 0 : (P0 + 2) % 3>{}, PF);  // unconditional (see the top of the file)
      __syncthreads();
      float p[V + 6], cs[V + 4], a[V], o[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) p[k] = lp[b][xi][w * V + k][lane];
#pragma unroll
      for (int k = 0; k < V + 4; ++k) cs[k] = lc[b][xi][w * V + 1 + k][lane];
      // sweep along the segment axis (second for even, first for odd)
      sweep_segment<V>(p, cs, a, flag);
      // sweep along the march axis (even: last; odd: second)
      march_step<V, P0>(ra, r1, re, rc, a, cm, o);
      if (t >= 6) {
        const unsigned qo = unsigned(pw.p[0]) * mstr;
        if (!EVEN)  // all lanes: the halo lanes feed the output lanes' neighbours
#pragma unroll
          for (int j = 0; j < V; ++j) o[j] = xsweep_lanes(o[j], cxo[j]);  // last sweep (x)
        if (lane_out) {
          const int rows_left = ns - s0;
#pragma unroll
          for (int j = 0; j < V; ++j)
            if (j < rows_left) st_vs(out, orow[j], qo, o[j]);
        }
      }
      pw.advance();
    };
    for (int t = 0; t < iters; t += 3) {
      body(std::integral_constant<int, 0>{}, t);
      if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
      if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
    }
    // the next run's first LDS writes must not meet this run's last reads
    __syncthreads();
  }
  if (over) *flag = 1;
}

// The persistent march's group shape: V = 4 rows per wave, W = 4 waves per
// window (16-row groups), WX = 3 windows per workgroup (12 waves).
constexpr int kWpV = 4, kWpW = 4, kWpWX = 3;

template <bool EVEN, int V, int W, int WX, int PF>
hipError_t launch_wp_t(const Geo& g, const float* phi, const float* u, float* out, int* flag,
                       hipStream_t st, int shape) {
  auto kern = k_cec3d_wp<EVEN, V, W, WX, PF>;
  constexpr int S = V * W;
  const size_t n = (size_t)g.ncells;
  const int ns = EVEN ? g.ny : g.nz, nm = EVEN ? g.nz : g.ny;
  const int nwx = (g.nx + kWmUse - 1) / kWmUse;
  const long long total = (long long)((nwx + WX - 1) / WX) * ((ns + S - 1) / S) * nm;
  static int cus = 0, fit = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, kern, 64 * W * WX, 0) != hipSuccess ||
        fit < 1)
      fit = 1;
  }
  long long blocks;
  int span;
  if (shape < 0) {  // chunks of -shape planes, one per workgroup
    const int chunk = -shape;
    span = -chunk;
    blocks = total / nm * ((nm + chunk - 1) / chunk);
  } else {
    const int per_cu = shape > 0 ? min(shape, fit) : fit;
    blocks = (long long)cus * per_cu;
    // every workgroup marches at least 16 planes
    blocks = max(1LL, min(blocks, total / 16));
    span = int((total + blocks - 1) / blocks);
    blocks = (total + span - 1) / span;
  }
  hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * W * WX), 0, st, phi, u, u + n,
                     u + 2 * n, out, g, span, flag);
  return hipGetLastError();
}

// shape > 0: persistent, workgroups per CU; < 0: march chunks of -shape
// planes, one workgroup per chunk of a group; 0: persistent, as many as fit
// pf: planes loaded ahead of the march (1 or 2); wx: windows per workgroup
hipError_t launch_cec3d_wp(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc, int pf = 1, int wx = kWpWX) {
  auto go = [&](auto wxc) {
    constexpr int WXC = decltype(wxc)::value;
    if (pf == 2)
      return even ? launch_wp_t<true, kWpV, kWpW, WXC, 2>(g, phi, u, out, flag, st, lc.ychunk)
                  : launch_wp_t<false, kWpV, kWpW, WXC, 2>(g, phi, u, out, flag, st, lc.ychunk);
    return even ? launch_wp_t<true, kWpV, kWpW, WXC, 1>(g, phi, u, out, flag, st, lc.ychunk)
                : launch_wp_t<false, kWpV, kWpW, WXC, 1>(g, phi, u, out, flag, st, lc.ychunk);
  };
  if (wx == 1) return go(std::integral_constant<int, 1>{});
  if (wx == 2) return go(std::integral_constant<int, 2>{});
  return go(std::integral_constant<int, kWpWX>{});
}

// ---------------------------------------------------------------------------
// Aligned two-node window march (variant 14).  The shared-halo march of
// variant 8 laid out on x windows of 128 nodes that start on 512-byte
// boundaries: lane l holds nodes 2l and 2l+1 (8-byte loads and stores) and a
// window computes all 128 of its outputs, so no lane computes a node that
// another window stores.  The three nodes beyond each end of the window (its
// x halo) are loaded apart, by six lanes per row.  The x sweep runs across
// the lanes as in the other variants; it is wrong at the window's first and
// last three nodes, whose stencils reach into the halo, and those six outputs
// of a row are computed again by a packed set of edge lanes (one per row and
// edge node) from the row's two 9-node end segments, gathered in a small LDS
// area of the wave.  Both parities march along z over groups of S = V*W =
// 32 y rows (38 loaded): odd steps, whose order is z, y, x, run the z sweep
// first, along the march on every loaded row, then y across the rows and x
// last; their halo nodes also go through the z and y sweeps, one (row, node)
// per lane.  W = 8 waves, one workgroup per CU, march chunks of up to 128
// planes.  Per node the same FP32 operations as
// the other variants.  Needs an even nx (a lane's two nodes are adjacent in
// memory, also where the window wraps around the row).
// ---------------------------------------------------------------------------
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned b64_t __attribute__((ext_vector_type(2)));  // the 64-bit buffer builtins' type
__device__ __forceinline__ f32x2 ld2_vs(const float* field, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(based_rsrc(field, soff), voff, 0, 0));
}
__device__ __forceinline__ void st2_vs(float* field, unsigned voff, unsigned soff, f32x2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64_t, v), based_rsrc(field, soff), voff, 0, 0);
}

// Third-order sweep along x of a row held as two nodes per lane (lane l:
// nodes 2l and 2l+1): the same operations per node as xsweep_lanes.  Node
// 2l-1 is lane l-1's second node, node 2l+2 lane l+1's first; the results of
// the first and last three nodes of the window are not valid.
__device__ __forceinline__ void xsweep_pairs(float& a, float& b, float ca, float cb) {
  const Dep1 da = depart1(ca, nullptr), db = depart1(cb, nullptr);
  const float pma = from_below(b), ppb = from_above(a);
  const float p1a = lerp(a, da.ob_neg ? pma : b, da.f);
  const float p1b = lerp(b, db.ob_neg ? a : ppb, db.f);
  const float qma = from_below(p1b), qpb = from_above(p1a);
  const float ea = a - lerp(p1a, da.obr_pos ? p1b : qma, da.f);
  const float eb = b - lerp(p1b, db.obr_pos ? qpb : p1a, db.f);
  const float ema = from_below(eb), epb = from_above(ea);
  const float ba = da.ob_neg ? ema : eb, bb = db.ob_neg ? ea : epb;
  const float wa = fmaf(da.f, 1.f / 3.f, 1.f / 3.f), wb = fmaf(db.f, 1.f / 3.f, 1.f / 3.f);
  a = fmaf(0.5f, fmaf(wa, ba - ea, ea), p1a);
  b = fmaf(0.5f, fmaf(wb, bb - eb, eb), p1b);
}

constexpr int kWqV = 4, kWqW = 8, kWqN = 128;  // rows per wave, waves per window, window nodes

// Slot of a window-relative node in a row's end segments (24 floats: nodes
// -3..5 at 1..9, nodes 122..130 at 12..20; a lane's pair starts on an even
// slot).
__device__ __forceinline__ int end_slot(int node) { return node < 64 ? node + 4 : node - 110; }

template <bool EVEN, int V, int W>
__global__ __launch_bounds__(64 * W) void k_cec3d_wq(const float* __restrict__ phi,
                                                     const float* __restrict__ ux,
                                                     const float* __restrict__ uy,
                                                     const float* __restrict__ uz,
                                                     float* __restrict__ out, Geo g, int chunk,
                                                     int* flag) {
  constexpr int S = V * W, NR = S + 6, RW = (NR + W - 1) / W;
  constexpr int LW = kWqN + 8;         // LDS row: the window's nodes, then (odd) its 6 halo nodes
  constexpr int NE = RW > V ? RW : V;  // rows with end segments per wave
  constexpr int NC = EVEN ? 2 * V : 2 * RW;  // march columns per lane: output rows (even), loaded rows (odd)
  static_assert(6 * NE <= 64, "one edge lane per row and end node");
  __shared__ __align__(16) float lp[2][NR][LW];     // y sweep input (x-swept if even, z-swept if odd)
  __shared__ __align__(16) float lc[2][NR][LW];     // y Courant numbers
  __shared__ __align__(16) float es[W][NE][2][24];  // end segments: values, x Courant numbers
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int nwx = (nx + kWqN - 1) / kWqN, ngs = (ny + S - 1) / S, ng = nwx * ngs;
  const int blk = block_tile(1).x;  // XCD-mapped 1D grid
  if (blk >= ng * ((nz + chunk - 1) / chunk)) return;  // the whole workgroup
  const int ch = blk / ng, grp = blk - ch * ng;
  const int x0 = (grp % nwx) * kWqN, g0 = (grp / nwx) * S, s0 = g0 + w * V;
  const int m0 = ch * chunk, m1 = min(nz, m0 + chunk);
  const unsigned rowb = 4u * unsigned(nx), plb = 4u * unsigned(nx) * unsigned(ny);
  const float lamX = g.lam[0], lamY = g.lam[1], lamZ = g.lam[2];
  const int nld = min(RW, NR - w * RW);  // rows this wave loads: w*RW + k, k < nld
  // lane 6k + i serves row k of the wave and end node i: the window's nodes
  // 0..2 and 125..127 (edge nodes), halo nodes -3..-1 and 128..130; lanes
  // past the rows repeat the last row and their results go unused
  const int ek = min(lane / 6, NE - 1), ei = lane - 6 * (lane / 6);
  const int hnode = ei < 3 ? ei - 3 : kWqN + ei - 3;  // window-relative halo node
  const int enode = ei < 3 ? ei : kWqN - 6 + ei;      // window-relative edge node
  const unsigned vx = 4u * unsigned(wrapk(x0 + 2 * lane, nx));
  const unsigned hx = 4u * unsigned(wrapk(x0 + hnode, nx));
  // per-lane offsets within a z plane of the loaded rows (rows past the
  // wave's share repeat its last row: every wave issues the same loads, none
  // under a condition) and of the output rows
  unsigned lrow[RW], orow[V];
#pragma unroll
  for (int k = 0; k < RW; ++k)
    lrow[k] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(g0 - 3 + w * RW + min(k, nld - 1), ny))) * rowb;
#pragma unroll
  for (int j = 0; j < V; ++j)
    orow[j] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(s0 + j, ny))) * rowb;
  // the halo node's offsets in loaded row min(ek, nld - 1) and output row min(ek, V - 1)
  const unsigned hlrow = hx + unsigned(wrapk(g0 - 3 + w * RW + min(ek, nld - 1), ny)) * rowb;
  const unsigned horow = hx + unsigned(wrapk(s0 + min(ek, V - 1), ny)) * rowb;
  PlaneWin pw(m0 - 6, nz);  // planes m0 - 6 + t .. m0 - 1 + t at iteration t

  // Iteration t loads plane q = m0 - 3 + t and writes plane q - 3.  Even
  // steps sweep x on the loaded rows of plane q, y on its output rows, and z
  // along the march (plane q - 3 out).  Odd steps sweep z first, along the
  // march on the loaded rows (plane q - 3 out of the rings), then y and x on
  // plane q - 3, whose y and x velocities are loaded three planes late.
  f32x2 fp[RW], fa[RW], fs[RW];  // loaded rows: phi; even: x, y velocity; odd: z (plane q-1), y (q-3)
  f32x2 fm[V];                   // output rows: even: z velocity (q-1); odd: x velocity (q-3)
  float hp, ha, hs, hm;          // this lane's halo node: phi, and velocities as the rows'
  // ahead: iterations after the current one.  Part 1: what the first
  // sweep of the iteration needs (even: all); part 2 (odd): the y and x
  // velocities of plane q - 3, issued after the iteration's stores so that
  // their registers are not held through its y sweep.
  auto prefetch = [&](int ahead, int part) {
    const unsigned q = unsigned(pw.plane(3 + ahead)) * plb,
                   qm1 = unsigned(pw.plane(2 + ahead)) * plb, qo = unsigned(pw.plane(ahead)) * plb;
    if (part & 1) {
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        fp[k] = ld2_vs(phi, lrow[k], q);
        fa[k] = EVEN ? ld2_vs(ux, lrow[k], q) : ld2_vs(uz, lrow[k], qm1);
        if (EVEN) fs[k] = ld2_vs(uy, lrow[k], q);
      }
      if (EVEN)
#pragma unroll
        for (int j = 0; j < V; ++j) fm[j] = ld2_vs(uz, orow[j], qm1);
      hp = ld_vs(phi, hlrow, q);
      ha = EVEN ? ld_vs(ux, hlrow, q) : ld_vs(uz, hlrow, qm1);
    }
    if (!EVEN && (part & 2)) {
#pragma unroll
      for (int k = 0; k < RW; ++k) fs[k] = ld2_vs(uy, lrow[k], qo);
#pragma unroll
      for (int j = 0; j < V; ++j) fm[j] = ld2_vs(ux, orow[j], qo);
      hs = ld_vs(uy, hlrow, qo);
      hm = ld_vs(ux, horow, qo);
    }
  };

  // march rings (z): even: node 2l of output row j in column j, node 2l+1 in
  // column V + j; odd: the loaded rows likewise (RW for V), and the halo
  // node of lane 6k + i (loaded row k) in a ring of its own
  float ra[3][NC], r1[3][NC], re[3][NC], rc[3][NC];
  float hra[3][1], hr1[3][1], hre[3][1], hrc[3][1];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int j = 0; j < NC; ++j) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;
    hra[k][0] = hr1[k][0] = hre[k][0] = hrc[k][0] = 0.f;
  }

  const int iters = (m1 - m0) + 6;
  const bool lane_out = x0 + 2 * lane < nx;
  const bool end_lane = lane < 3 || lane >= 61;  // holds nodes of the end segments
  const int eslot = end_slot(2 * lane);
  const int hslot = end_slot(hnode), e0slot = end_slot(enode);
  bool over = false;
  // x sweep of the end nodes of rows 0..nrows-1 of the wave, from their end
  // segments (lane 6k + i: row k, edge node i); returns this lane's result
  auto edge_x = [&]() {
    float p[7], c[5], o[1];
#pragma unroll
    for (int i = 0; i < 7; ++i) p[i] = es[w][ek][0][e0slot - 3 + i];
#pragma unroll
    for (int i = 0; i < 5; ++i) c[i] = es[w][ek][1][e0slot - 2 + i];
    sweep_segment<1>(p, c, o, flag);
    return o[0];
  };
  prefetch(0, 3);
  auto body = [&](auto phase, int t) {
    constexpr int P0 = decltype(phase)::value;
    const int b = t & 1;
    if constexpr (EVEN) {
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        if (k < nld) {
          float va = fp[k].x, vb = fp[k].y;
          const float ca = fa[k].x * lamX, cb = fa[k].y * lamX;
          over |= over1(ca) | over1(cb);
          if (end_lane) {
            *reinterpret_cast<f32x2*>(&es[w][k][0][eslot]) = f32x2{va, vb};
            *reinterpret_cast<f32x2*>(&es[w][k][1][eslot]) = f32x2{ca, cb};
          }
          xsweep_pairs(va, vb, ca, cb);  // first sweep (x) of this row; its ends below
          const float sa = fs[k].x * lamY, sb = fs[k].y * lamY;
          over |= over1(sa) | over1(sb);
          *reinterpret_cast<f32x2*>(&lp[b][w * RW + k][2 * lane]) = f32x2{va, vb};
          *reinterpret_cast<f32x2*>(&lc[b][w * RW + k][2 * lane]) = f32x2{sa, sb};
        }
      }
      // the x sweep at the first and last three nodes of each loaded row
      if (lane < 6 * nld) {
        es[w][ek][0][hslot] = hp;
        es[w][ek][1][hslot] = ha * lamX;
      }
      const float eo = edge_x();
      if (lane < 6 * nld) lp[b][w * RW + ek][enode] = eo;
    } else {
      // first sweep (z) along the march on the loaded rows: plane q - 3 out
      float za[NC], zc[NC], zo[NC];
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        za[k] = fp[k].x;
        za[RW + k] = fp[k].y;
        zc[k] = fa[k].x * lamZ;
        zc[RW + k] = fa[k].y * lamZ;
        over |= over1(zc[k]) | over1(zc[RW + k]);
      }
      march_step<NC, P0>(ra, r1, re, rc, za, zc, zo);
      float hza[1] = {hp}, hzc[1] = {ha * lamZ}, hzo[1];
      march_step<1, P0>(hra, hr1, hre, hrc, hza, hzc, hzo);
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        if (k < nld) {
          const float sa = fs[k].x * lamY, sb = fs[k].y * lamY;
          over |= over1(sa) | over1(sb);
          *reinterpret_cast<f32x2*>(&lp[b][w * RW + k][2 * lane]) = f32x2{zo[k], zo[RW + k]};
          *reinterpret_cast<f32x2*>(&lc[b][w * RW + k][2 * lane]) = f32x2{sa, sb};
        }
      }
      if (lane < 6 * nld) {  // the halo nodes' y sweep inputs
        lp[b][w * RW + ek][kWqN + ei] = hzo[0];
        lc[b][w * RW + ek][kWqN + ei] = hs * lamY;
      }
    }
    float cm[2 * V];  // even: z Courant numbers of plane q-1; odd: x Courant numbers of plane q-3
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float lm = EVEN ? lamZ : lamX;
      cm[j] = fm[j].x * lm;
      cm[V + j] = fm[j].y * lm;
      over |= over1(cm[j]) | over1(cm[V + j]);
    }
    const float hcx = EVEN ? 0.f : hm * lamX;
    prefetch(1, 1);  // unconditional (see the top of the file)
    __syncthreads();
    float a[2 * V];  // y sweep (second) of the output rows
    {
      float pa[V + 6], pb[V + 6], csa[V + 4], csb[V + 4], aa[V], ab[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) {
        const f32x2 v = *reinterpret_cast<const f32x2*>(&lp[b][w * V + k][2 * lane]);
        pa[k] = v.x;
        pb[k] = v.y;
      }
#pragma unroll
      for (int k = 0; k < V + 4; ++k) {
        const f32x2 c = *reinterpret_cast<const f32x2*>(&lc[b][w * V + 1 + k][2 * lane]);
        csa[k] = c.x;
        csb[k] = c.y;
      }
      sweep_segment<V>(pa, csa, aa, flag);
      sweep_segment<V>(pb, csb, ab, flag);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        a[j] = aa[j];
        a[V + j] = ab[j];
      }
    }
    float o[2 * V];
    float yh = 0.f;
    if constexpr (EVEN) {
      march_step<NC, P0>(ra, r1, re, rc, a, cm, o);  // last sweep (z): plane q - 3 out
    } else {
#pragma unroll
      for (int j = 0; j < 2 * V; ++j) o[j] = a[j];
      // the y sweep at the halo node of lane 6j + i (output row j)
      float ph[7], chh[5], ah[1];
      const int r0 = w * V + min(ek, V - 1);
#pragma unroll
      for (int i = 0; i < 7; ++i) ph[i] = lp[b][r0 + i][kWqN + ei];
#pragma unroll
      for (int i = 0; i < 5; ++i) chh[i] = lc[b][r0 + 1 + i][kWqN + ei];
      sweep_segment<1>(ph, chh, ah, flag);
      yh = ah[0];
    }
    if (t >= 6) {
      const unsigned qo = unsigned(pw.p[0]) * plb;
      float xa[V], xb[V];
#pragma unroll
      for (int j = 0; j < V; ++j) {
        xa[j] = o[j];
        xb[j] = o[V + j];
      }
      if (!EVEN) {  // last sweep (x), the ends from the edge lanes
#pragma unroll
        for (int j = 0; j < V; ++j) {
          if (end_lane) {
            *reinterpret_cast<f32x2*>(&es[w][j][0][eslot]) = f32x2{xa[j], xb[j]};
            *reinterpret_cast<f32x2*>(&es[w][j][1][eslot]) = f32x2{cm[j], cm[V + j]};
          }
          xsweep_pairs(xa[j], xb[j], cm[j], cm[V + j]);
        }
        if (lane < 6 * V) {
          es[w][ek][0][hslot] = yh;
          es[w][ek][1][hslot] = hcx;
        }
        const int eoi = __builtin_bit_cast(int, edge_x());
        // lane 0 takes nodes 0 and 1, lane 1 node 2, lane 62 node 125, lane
        // 63 nodes 126 and 127 from the edge lanes 6j + 0..5
        const int sa = lane == 0 ? 0 : lane == 1 ? 2 : 4, sb = lane == 0 ? 1 : lane == 62 ? 3 : 5;
        const bool ta = lane == 0 || lane == 1 || lane == 63, tb = lane == 0 || lane == 62 || lane == 63;
#pragma unroll
        for (int j = 0; j < V; ++j) {
          const float va = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(4 * (6 * j + sa), eoi));
          const float vb = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(4 * (6 * j + sb), eoi));
          if (ta) xa[j] = va;
          if (tb) xb[j] = vb;
        }
      }
      if (lane_out) {
        const int rows_left = ny - s0;
#pragma unroll
        for (int j = 0; j < V; ++j)
          if (j < rows_left) st2_vs(out, orow[j], qo, f32x2{xa[j], xb[j]});
      }
    }
    if (!EVEN) prefetch(1, 2);
    pw.advance();
  };
  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

// Launch of the aligned two-node march: shape < 0 gives the march chunk
// (-shape planes); 0 the longest of 128, 64, 32 and 16 planes that still
// gives every CU a workgroup.
template <bool EVEN>
hipError_t launch_wq_t(const Geo& g, const float* phi, const float* u, float* out, int* flag,
                       hipStream_t st, int shape) {
  constexpr int V = kWqV, W = kWqW, S = V * W;
  const size_t n = (size_t)g.ncells;
  const int nm = g.nz;  // both parities march along z
  const long long groups = (long long)((g.nx + kWqN - 1) / kWqN) * ((g.ny + S - 1) / S);
  int chunk = shape < 0 ? -shape : 0;
  if (chunk <= 0) {
    static int cus = 0;
    if (!cus) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    }
    chunk = 16;
    for (int c : {128, 64, 32})
      if (groups * ((nm + c - 1) / c) >= cus) {
        chunk = c;
        break;
      }
  }
  const long long blocks = groups * ((nm + chunk - 1) / chunk);
  hipLaunchKernelGGL((k_cec3d_wq<EVEN, V, W>), dim3(unsigned(blocks)), dim3(64 * W), 0, st, phi, u,
                     u + n, u + 2 * n, out, g, chunk, flag);
  return hipGetLastError();
}
hipError_t launch_cec3d_wq(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc) {
  if (g.nx % 2) return hipErrorInvalidValue;
  return even ? launch_wq_t<true>(g, phi, u, out, flag, st, lc.ychunk)
              : launch_wq_t<false>(g, phi, u, out, flag, st, lc.ychunk);
}

// ---------------------------------------------------------------------------
// Several fields sharing one velocity (K per launch): the shared-halo window
// march of variant 7 with the velocity loaded once per tile for all K
// fields.  Per march plane a workgroup loads the velocity rows its tile
// needs and forms the Courant numbers once; then, field after field, it
// loads the field's rows, runs its first sweep, exchanges the rows through
// LDS (one barrier per field and plane, the LDS buffers alternating along
// the sequence of fields and planes), and runs the segment sweep and the
// march step on that field's own register pipeline.  A field's value at a
// node goes through the same FP32 operations as in the single-field kernels,
// so every field ends bit for bit as if advanced alone.
// ---------------------------------------------------------------------------
constexpr int kMfMax = 4;
struct MfFields {
  const float* in[kMfMax];
  float* out[kMfMax];
};

template <bool EVEN, int V, int W, int WX, int K>
__global__ __launch_bounds__(64 * W * WX) void k_cec3d_mf(MfFields fl, const float* __restrict__ ux,
                                                          const float* __restrict__ uy,
                                                          const float* __restrict__ uz, Geo g,
                                                          int chunk, int* flag) {
  constexpr int S = V * W, NR = S + 6, RW = (NR + W - 1) / W, kAll = NR - (W - 1) * RW;
  __shared__ float lp[2][WX][NR][64];  // a field's segment sweep input (x-swept if even)
  __shared__ float lc[2][WX][NR][64];  // segment-axis Courant numbers of a plane
  const int lane = threadIdx.x & 63, xi = (threadIdx.x >> 6) % WX, w = (threadIdx.x >> 6) / WX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ns = EVEN ? ny : nz, nm = EVEN ? nz : ny;
  const int nwx = (nx + kWmUse - 1) / kWmUse, ngx = (nwx + WX - 1) / WX, ngs = (ns + S - 1) / S;
  const int nch = (nm + chunk - 1) / chunk;
  const int blk = block_tile(1).x;  // 1D grid, XCD-mapped
  if (blk >= ngx * ngs * nch) return;  // the whole workgroup
  const int wx0 = (blk % ngx) * WX, gs = (blk / ngx) % ngs, ch = blk / (ngx * ngs);
  const bool wx_ok = wx0 + xi < nwx;  // the same for the whole wave
  const int wx = min(wx0 + xi, nwx - 1);
  const unsigned vx = 4u * unsigned(wrapk(wx * kWmUse - 3 + lane, nx));
  const unsigned rowb = 4u * unsigned(nx), plb = 4u * unsigned(nx) * unsigned(ny);
  const unsigned sstr = EVEN ? rowb : plb, mstr = EVEN ? plb : rowb;
  const int g0 = gs * S, s0 = g0 + w * V, m0 = ch * chunk, m1 = min(m0 + chunk, nm);
  const int nld = min(RW, NR - w * RW);
  unsigned loff[RW], ooff[V];
#pragma unroll
  for (int k = 0; k < RW; ++k)
    loff[k] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(g0 - 3 + w * RW + k, ns))) * sstr;
#pragma unroll
  for (int j = 0; j < V; ++j)
    ooff[j] = vx + unsigned(__builtin_amdgcn_readfirstlane(wrapk(s0 + j, ns))) * sstr;
  const float* rS = EVEN ? uy : uz;  // segment-axis velocity
  const float* rM = EVEN ? uz : uy;  // march-axis velocity
  const float lamX = g.lam[0], lamS = EVEN ? g.lam[1] : g.lam[2], lamM = EVEN ? g.lam[2] : g.lam[1];
  PlaneWin pw(m0 - 6, nm);  // planes m0 - 6 + t .. m0 - 2 + t at iteration t

  float fp[K][RW], fa[RW], fs[RW];  // fields, x velocity (even), segment velocity: loaded rows
  float fm[V], fx[V];               // march velocity of plane q-1; odd: x velocity of the output plane
  auto prefetch = [&](int ahead) {  // 0: iteration t; 1: iteration t + 1
    const unsigned q = unsigned(pw.p[3 + ahead]) * mstr, qm1 = unsigned(pw.p[2 + ahead]) * mstr,
                   qo = unsigned(pw.p[ahead]) * mstr;
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      if (k < kAll || k < nld) {
        if (EVEN) fa[k] = ld_vs(ux, loff[k], q);
        fs[k] = ld_vs(rS, loff[k], q);
#pragma unroll
        for (int f = 0; f < K; ++f) fp[f][k] = ld_vs(fl.in[f], loff[k], q);
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      fm[j] = ld_vs(rM, ooff[j], qm1);
      if (!EVEN) fx[j] = ld_vs(ux, ooff[j], qo);
    }
  };

  // per field: rings of the march pipeline; the Courant ring is shared
  float ra[K][3][V], r1[K][3][V], re[K][3][V], rc[3][V];
#pragma unroll
  for (int j = 0; j < V; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rc[k][j] = 0.f;
#pragma unroll
      for (int f = 0; f < K; ++f) ra[f][k][j] = r1[f][k][j] = re[f][k][j] = 0.f;
    }

  const int iters = (m1 - m0) + 6;
  const bool lane_out = lane >= 3 && lane < 61 && wx * kWmUse + lane - 3 < nx;
  bool over = false;
  if (wx_ok) prefetch(0);
  auto body = [&](auto phase, int t) {
    constexpr int P0 = decltype(phase)::value;
    if (!wx_ok) {  // a window past the row's end: barriers only
#pragma unroll
      for (int f = 0; f < K; ++f) __syncthreads();
      return;
    }
    // the velocity part of this plane, shared by the fields
    float cxr[RW], cm[V], cxo[V];
    float pv[K][RW];
#pragma unroll
    for (int k = 0; k < RW; ++k) {
      if (k < kAll || k < nld) {
        if (EVEN) {
          cxr[k] = fa[k] * lamX;
          over |= over1(cxr[k]);
        }
        const float c = fs[k] * lamS;
        over |= over1(c);
        lc[t & 1][xi][w * RW + k][lane] = c;
#pragma unroll
        for (int f = 0; f < K; ++f) pv[f][k] = fp[f][k];
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      cm[j] = fm[j] * lamM;
      over |= over1(cm[j]);
      cxo[j] = EVEN ? 0.f : fx[j] * lamX;
      if (!EVEN) over |= over1(cxo[j]);
    }
    prefetch(1);  // unconditional (see the top of the file)
#pragma unroll
    for (int f = 0; f < K; ++f) {
      const int bf = (t * K + f) & 1;
#pragma unroll
      for (int k = 0; k < RW; ++k) {
        if (k < kAll || k < nld) {
          float v = pv[f][k];
          if (EVEN) v = xsweep_lanes(v, cxr[k]);  // first sweep (x) of this row
          lp[bf][xi][w * RW + k][lane] = v;
        }
      }
      __syncthreads();
      float p[V + 6], cs[V + 4], a[V], o[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) p[k] = lp[bf][xi][w * V + k][lane];
#pragma unroll
      for (int k = 0; k < V + 4; ++k) cs[k] = lc[t & 1][xi][w * V + 1 + k][lane];
      // sweep along the segment axis (second for even, first for odd)
      sweep_segment<V>(p, cs, a, flag);
      // sweep along the march axis (even: last; odd: second); the Courant
      // ring advances with the first field only
      if (f == 0) {
        march_step<V, P0>(ra[0], r1[0], re[0], rc, a, cm, o);
      } else {
        float rcf[3][V];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int j = 0; j < V; ++j) rcf[k][j] = rc[k][j];
        // rc already holds this plane's entry: march_step writes the same
        // value into its own copy
        march_step<V, P0>(ra[f], r1[f], re[f], rcf, a, cm, o);
      }
      if (t >= 6) {
        const unsigned qo = unsigned(pw.p[0]) * mstr;
        if (!EVEN)
#pragma unroll
          for (int j = 0; j < V; ++j) o[j] = xsweep_lanes(o[j], cxo[j]);  // last sweep (x)
        store_rows<V>(fl.out[f], ooff, qo, o, lane_out, ns - s0);
      }
    }
    pw.advance();
  };
  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

// Multi-field launch shapes: (V, W, WX) per field count.
template <int K>
struct MfShape;
template <>
struct MfShape<2> {
  static constexpr int V = 4, W = 4, WX = 3;
};
template <>
struct MfShape<4> {
  static constexpr int V = 4, W = 4, WX = 2;
};

template <int K>
hipError_t launch_mf_k(bool even, const Geo& g, const MfFields& fl, const float* u, int* flag,
                       hipStream_t st, int chunk) {
  using Sh = MfShape<K>;
  constexpr int S = Sh::V * Sh::W;
  const size_t n = (size_t)g.ncells;
  const int ns = even ? g.ny : g.nz, nm = even ? g.nz : g.ny;
  const long long groups =
      (long long)(((g.nx + kWmUse - 1) / kWmUse + Sh::WX - 1) / Sh::WX) * ((ns + S - 1) / S);
  if (chunk <= 0) {
    chunk = 16;
    for (int c : {64, 32})
      if (groups * ((nm + c - 1) / c) >= 512) { chunk = c; break; }
  }
  dim3 grid(unsigned(groups * ((nm + chunk - 1) / chunk)));
  if (even)
    hipLaunchKernelGGL((k_cec3d_mf<true, Sh::V, Sh::W, Sh::WX, K>), grid, dim3(64 * Sh::W * Sh::WX),
                       0, st, fl, u, u + n, u + 2 * n, g, chunk, flag);
  else
    hipLaunchKernelGGL((k_cec3d_mf<false, Sh::V, Sh::W, Sh::WX, K>), grid, dim3(64 * Sh::W * Sh::WX),
                       0, st, fl, u, u + n, u + 2 * n, g, chunk, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming variant: 512-thread workgroups; every plane of phi and of the
// Courant numbers reaches LDS through direct global-to-LDS loads (no
// registers, no per-load address arithmetic: a per-plane base in scalar
// registers plus per-lane 32-bit offsets computed once).  phi and the
// first sweep's velocity are double-buffered and fetched a whole plane
// ahead; the y and last-sweep velocities are fetched one phase ahead.  The
// first and last sweeps run as register segments, the y sweep as the
// register pipeline.  Four barriers per plane.
// ---------------------------------------------------------------------------
constexpr int kT4 = 512;

template <bool EVEN>
struct V4Shape {
  static constexpr int H = 3, TX = 64, TZ = 16;
  static constexpr int W = TX + 2 * H, HZ = TZ + 2 * H, NP = W * HZ;
  static constexpr int TA = EVEN ? TX : TZ, TB = EVEN ? TZ : TX;
  static constexpr int SA = EVEN ? 1 : W, SB = EVEN ? W : 1;
  // y region: x-fastest rectangle [YX0, YX0+YW) x [YZ0, YZ0+YH)
  static constexpr int YX0 = EVEN ? 0 : -H, YW = EVEN ? TX : TX + 2 * H;
  static constexpr int YZ0 = EVEN ? -H : 0, YH = EVEN ? TZ + 2 * H : TZ;
  static constexpr int NY = YW * YH;
  static constexpr int KY = (NY + kT4 - 1) / kT4;  // y columns per thread
  static constexpr int V = 8;
  static constexpr int NS1 = TA / V, N1 = (TB + 2 * H) * NS1;
  static constexpr int NS2 = TB / V, N2 = TA * NS2;
  // LDS chunks of 64 floats: the padded plane, and the y region
  static constexpr int CP = (NP + 63) / 64;
  static constexpr int CPW = (CP + kT4 / 64 - 1) / (kT4 / 64);  // per wave
  static constexpr int CYc = (NY + 63) / 64;
  static constexpr int CYW = (CYc + kT4 / 64 - 1) / (kT4 / 64);
  static_assert(N1 <= kT4 && N2 <= kT4, "one segment per thread");
};

template <bool EVEN>
__device__ __forceinline__ int v4_lidx(int x, int z) {
  using S = V4Shape<EVEN>;
  return (z + S::H) * S::W + (x + S::H);
}

typedef __attribute__((address_space(3))) void lds_void;

// Direct global -> LDS load of one float per lane into lds_chunk[lane].
__device__ __forceinline__ void g2l(const float* base, unsigned byte_off, float* lds_chunk) {
  __builtin_amdgcn_global_load_lds(
      reinterpret_cast<const void*>(reinterpret_cast<const char*>(base) + byte_off),
      (lds_void*)(lds_chunk), 4, 0, 0);
}

// One tile of one problem for the streaming variant.  umask is ~0u for a
// velocity field and 0 for a uniform velocity (u points at one value per
// axis; every lane then reads that value).
struct Tile {
  const float* phi;
  float* out;
  const float* u[3];
  unsigned umask;
  int nx, ny, nz;
  float lam[3];
  int x0, z0, y0, y1;
};

struct V4Lds {
  float P[2][V4Shape<true>::NP];   // phi, double-buffered by plane parity
  float UA[2][V4Shape<true>::NP];  // first-sweep velocity (raw), double-buffered
  float UY[V4Shape<true>::NY > V4Shape<false>::NY ? V4Shape<true>::NY : V4Shape<false>::NY];
  float UB[V4Shape<true>::NP];     // last-sweep velocity at the output plane (raw)
  float AO[V4Shape<true>::NP];     // first-sweep output
  float YO[V4Shape<true>::NP];     // y-sweep output
};

template <bool EVEN>
__device__ __forceinline__ void cec3d_tile_v4(const Tile& T, V4Lds& L, int* flag) {
  using S = V4Shape<EVEN>;
  constexpr int H = S::H, TA = S::TA, SA = S::SA, SB = S::SB, V = S::V, KY = S::KY;
  static_assert(V4Shape<true>::NP == V4Shape<false>::NP, "same padded plane");
  auto& P = L.P;
  auto& UA = L.UA;
  float* UY = L.UY;
  float* UB = L.UB;
  float* AO = L.AO;
  float* YO = L.YO;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int x0 = T.x0, z0 = T.z0, y0 = T.y0, y1 = T.y1;
  const int nx = T.nx, ny = T.ny, nz = T.nz;
  const unsigned nxy = unsigned(nx) * unsigned(ny);
  const float* phi = T.phi;
  float* out = T.out;
  const float* uA = EVEN ? T.u[0] : T.u[2];
  const float* uB = EVEN ? T.u[2] : T.u[0];
  const float* uy = T.u[1];
  const unsigned um = T.umask;
  const float lamA = EVEN ? T.lam[0] : T.lam[2];
  const float lamB = EVEN ? T.lam[2] : T.lam[0];
  const float lamY = T.lam[1];

  // byte offsets (x-z part) of this lane's element in each chunk it loads
  unsigned pofs[S::CPW], yofs[S::CYW];
#pragma unroll
  for (int k = 0; k < S::CPW; ++k) {
    const int e = min((wave + k * (kT4 / 64)) * 64 + lane, S::NP - 1);
    const int z = e / S::W - H, x = e % S::W - H;
    pofs[k] = 4u * (unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz)));
  }
#pragma unroll
  for (int k = 0; k < S::CYW; ++k) {
    const int e = min((wave + k * (kT4 / 64)) * 64 + lane, S::NY - 1);
    const int z = S::YZ0 + e / S::YW, x = S::YX0 + e % S::YW;
    yofs[k] = 4u * (unsigned(wrap1(x0 + x, nx)) + nxy * unsigned(wrap1(z0 + z, nz)));
  }
  // padded-plane position of y-region element e (for UB, AO, YO)
  auto ypos = [&](int e) {
    const int z = S::YZ0 + e / S::YW, x = S::YX0 + e % S::YW;
    return v4_lidx<EVEN>(x, z);
  };
  const unsigned rowb = 4u * unsigned(nx);  // bytes per y step

  // issue the loads of one padded plane (phi + first-sweep velocity) at y = q
  auto fetch_plane = [&](int q, int buf) {
    const unsigned qb = unsigned(wrap1(q, ny)) * rowb;
#pragma unroll
    for (int k = 0; k < S::CPW; ++k) {
      const int ch = wave + k * (kT4 / 64);
      if (ch >= S::CP) break;
      if (ch * 64 + lane < S::NP) {
        g2l(phi, pofs[k] + qb, &P[buf][ch * 64]);
        g2l(uA, (pofs[k] + qb) & um, &UA[buf][ch * 64]);
      }
    }
  };
  // y velocity of plane q into UY (y-region order)
  auto fetch_uy = [&](int q) {
    const unsigned qb = unsigned(wrap1(q, ny)) * rowb;
#pragma unroll
    for (int k = 0; k < S::CYW; ++k) {
      const int ch = wave + k * (kT4 / 64);
      if (ch >= S::CYc) break;
      if (ch * 64 + lane < S::NY) g2l(uy, (yofs[k] + qb) & um, &UY[ch * 64]);
    }
  };
  // last-sweep velocity of plane q into UB at the y-region positions: the
  // region is whole padded rows (odd) or 64-wide rows (even), so each chunk
  // of 64 consecutive region elements is 64 consecutive LDS floats
  auto fetch_ub = [&](int q) {
    const unsigned qb = unsigned(wrap1(q, ny)) * rowb;
#pragma unroll
    for (int k = 0; k < S::CYW; ++k) {
      const int ch = wave + k * (kT4 / 64);
      if (ch >= S::CYc) break;
      if (ch * 64 + lane < S::NY) g2l(uB, (yofs[k] + qb) & um, &UB[ypos(ch * 64)]);
    }
  };
  static_assert(EVEN ? (S::YW == 64) : (S::YW == S::W), "y-region chunks are contiguous in LDS");

  // segment items
  const bool has1 = tid < S::N1, has2 = tid < S::N2;
  const int i1 = EVEN ? v4_lidx<EVEN>((tid % S::NS1) * V, tid / S::NS1 - H)
                      : v4_lidx<EVEN>(tid / S::NS1 - H, (tid % S::NS1) * V);
  const int la2 = EVEN ? tid % TA : tid / S::NS2;
  const int sb2 = EVEN ? tid / TA : tid % S::NS2;
  const int i2 = EVEN ? v4_lidx<EVEN>(la2, sb2 * V) : v4_lidx<EVEN>(sb2 * V, la2);
  const int ox2 = EVEN ? la2 : sb2 * V, oz2 = EVEN ? sb2 * V : la2;

  int ycol[KY];
#pragma unroll
  for (int j = 0; j < KY; ++j) ycol[j] = ypos(min(tid + j * kT4, S::NY - 1));
  auto yvalid = [&](int j) { return KY * kT4 == S::NY || tid + j * kT4 < S::NY; };

  float ra[3][KY], r1[3][KY], re[3][KY], rc[3][KY];
#pragma unroll
  for (int j = 0; j < KY; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) ra[k][j] = r1[k][j] = re[k][j] = rc[k][j] = 0.f;

  const int iters = (y1 - y0) + 2 * H;
  bool over = false;
  __syncthreads();  // LDS of a previous tile is no longer read
  fetch_plane(y0 - H, 0);
  fetch_uy(y0 - H - 1);
  fetch_ub(y0 - 2 * H);

  auto body = [&](auto phase, int t) {
    constexpr int p0 = decltype(phase)::value;  // t % 3
    constexpr int p1 = (p0 + 2) % 3;            // (t - 1) % 3
    constexpr int p2 = (p0 + 1) % 3;            // (t - 2) % 3
    constexpr int p3 = p0;                      // (t - 3) % 3
    const bool emit = t >= 2 * H;
    const int buf = t & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of plane t have landed
    __syncthreads();
    if (t + 1 < iters) fetch_plane(y0 - H + t + 1, buf ^ 1);
    // 1. first sweep, one segment per thread
    if (has1) {
      float p[V + 6], c[V + 4], o[V];
#pragma unroll
      for (int k = 0; k < V + 6; ++k) p[k] = P[buf][i1 + (k - 3) * SA];
#pragma unroll
      for (int k = 0; k < V + 4; ++k) {
        c[k] = UA[buf][i1 + (k - 2) * SA] * lamA;
        over |= over1(c[k]);
      }
      sweep_segment<V>(p, c, o, flag);
#pragma unroll
      for (int k = 0; k < V; ++k) AO[i1 + k * SA] = o[k];
    }
    __syncthreads();
    // 2. y sweep as a pipeline along the march
    float cy[KY];
#pragma unroll
    for (int j = 0; j < KY; ++j) cy[j] = UY[min(tid + j * kT4, S::NY - 1)] * lamY;
#pragma unroll
    for (int j = 0; j < KY; ++j) {
      if (!yvalid(j)) continue;
      over |= over1(cy[j]);
      const int i = ycol[j];
      ra[p0][j] = AO[i];
      rc[p1][j] = cy[j];
      Dep1 d = depart1(rc[p1][j], flag);
      r1[p1][j] = lerp(ra[p1][j], d.ob_neg ? ra[p2][j] : ra[p0][j], d.f);
      d = depart1(rc[p2][j], flag);
      re[p2][j] = ra[p2][j] - lerp(r1[p2][j], d.obr_pos ? r1[p1][j] : r1[p3][j], d.f);
      d = depart1(rc[p3][j], flag);
      const float ea = re[p3][j];
      const float eb = d.ob_neg ? re[p1][j] : re[p2][j];
      const float w = fmaf(d.f, 1.f / 3.f, 1.f / 3.f);
      YO[i] = fmaf(0.5f, fmaf(w, eb - ea, ea), r1[p3][j]);
    }
    __syncthreads();
    if (t + 1 < iters) fetch_uy(y0 - H + t);  // y velocity of plane t, used at t + 1
    if (emit) {
      // 3. last sweep, one segment per thread, stored to HBM at plane t - 6
      if (has2) {
        float p[V + 6], c[V + 4], o[V];
#pragma unroll
        for (int k = 0; k < V + 6; ++k) p[k] = YO[i2 + (k - 3) * SB];
#pragma unroll
        for (int k = 0; k < V + 4; ++k) {
          c[k] = UB[i2 + (k - 2) * SB] * lamB;
          over |= over1(c[k]);
        }
        sweep_segment<V>(p, c, o, flag);
        const unsigned yo = unsigned(y0 + t - 2 * H) * unsigned(nx);
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const int x = x0 + ox2 + (EVEN ? 0 : k), z = z0 + oz2 + (EVEN ? k : 0);
          if (x < nx && z < nz) out[unsigned(x) + yo + nxy * unsigned(z)] = o[k];
        }
      }
    }
    __syncthreads();  // UB and YO are rewritten next
    if (t + 1 < iters) fetch_ub(y0 + t + 1 - 2 * H);
  };

  for (int t = 0; t < iters; t += 3) {
    body(std::integral_constant<int, 0>{}, t);
    if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 < iters) body(std::integral_constant<int, 2>{}, t + 2);
  }
  if (over) *flag = 1;
}

template <bool EVEN>
__global__ __launch_bounds__(kT4, 4) void k_cec3d_v4(const float* __restrict__ phi,
                                                     const float* __restrict__ ux,
                                                     const float* __restrict__ uy,
                                                     const float* __restrict__ uz,
                                                     float* __restrict__ out, Geo g, int ychunk, int swz,
                                                     int* flag) {
  __shared__ V4Lds L;
  Tile T;
  T.phi = phi;
  T.out = out;
  T.u[0] = ux;
  T.u[1] = uy;
  T.u[2] = uz;
  T.umask = ~0u;
  T.nx = g.nx;
  T.ny = g.ny;
  T.nz = g.nz;
  T.lam[0] = g.lam[0];
  T.lam[1] = g.lam[1];
  T.lam[2] = g.lam[2];
  const int3 bt = block_tile(swz);
  T.x0 = bt.x * V4Shape<EVEN>::TX;
  T.z0 = bt.y * V4Shape<EVEN>::TZ;
  T.y0 = bt.z * ychunk;
  T.y1 = min(T.y0 + ychunk, g.ny);
  cec3d_tile_v4<EVEN>(T, L, flag);
}

// ---------------------------------------------------------------------------
// Batched step: many problems (fields sharing a velocity, or independent
// grids with a uniform velocity) advanced by one third-order step in one
// persistent launch.  A workgroup takes items blockIdx.x, +gridDim.x, ...;
// an item is one tile (x tile, z tile, y chunk) of one problem.
// ---------------------------------------------------------------------------
template <bool EVEN>
__global__ __launch_bounds__(kT4, 4) void k_cec3d_batch(const BatchProblem* __restrict__ probs,
                                                        const int4* __restrict__ items,
                                                        int nitems, int parity, int* flag) {
  __shared__ V4Lds L;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 item = items[it];
    if (item.x < 0) continue;  // alignment hole (uniform across the block)
    const BatchProblem& B = probs[item.x];
    Tile T;
    T.phi = B.buf[parity];
    T.out = B.buf[parity ^ 1];
    T.u[0] = B.u[0];
    T.u[1] = B.u[1];
    T.u[2] = B.u[2];
    T.umask = B.umask;
    T.nx = B.n[0];
    T.ny = B.n[1];
    T.nz = B.n[2];
    T.lam[0] = B.lam[0];
    T.lam[1] = B.lam[1];
    T.lam[2] = B.lam[2];
    T.x0 = item.y * V4Shape<EVEN>::TX;
    T.z0 = item.z * V4Shape<EVEN>::TZ;
    T.y0 = item.w * B.ychunk;
    T.y1 = min(T.y0 + B.ychunk, B.n[1]);
    cec3d_tile_v4<EVEN>(T, L, flag);
  }
}

}  // namespace

hipError_t launch_cec3d_v4(bool even, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, Cec3dLaunch lc) {
  const size_t n = (size_t)g.ncells;
  const int ychunk = lc.ychunk > 0 ? lc.ychunk : cec3d_default_ychunk(g);
  dim3 grid((g.nx + 63) / 64, (g.nz + 15) / 16, (g.ny + ychunk - 1) / ychunk);
  if (even)
    hipLaunchKernelGGL(k_cec3d_v4<true>, grid, dim3(kT4), 0, st, phi, u, u + n, u + 2 * n, out, g,
                       ychunk, lc.swizzle, flag);
  else
    hipLaunchKernelGGL(k_cec3d_v4<false>, grid, dim3(kT4), 0, st, phi, u, u + n, u + 2 * n, out, g,
                       ychunk, lc.swizzle, flag);
  return hipGetLastError();
}

hipError_t launch_cec3d_batch(bool even, const BatchProblem* probs, const int4* items, int nitems,
                              int parity, int grid, int* flag, hipStream_t st) {
  if (even)
    hipLaunchKernelGGL(k_cec3d_batch<true>, dim3(grid), dim3(kT4), 0, st, probs, items, nitems,
                       parity, flag);
  else
    hipLaunchKernelGGL(k_cec3d_batch<false>, dim3(grid), dim3(kT4), 0, st, probs, items, nitems,
                       parity, flag);
  return hipGetLastError();
}

// buf[0] = buf[1] for every problem (after an odd number of steps).
__global__ __launch_bounds__(256) void k_batch_copy_back(const BatchProblem* __restrict__ probs) {
  const BatchProblem& B = probs[blockIdx.y];
  const size_t n = size_t(B.n[0]) * B.n[1] * B.n[2];
  const float* src = B.buf[1];
  float* dst = B.buf[0];
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    dst[i] = src[i];
}

hipError_t launch_batch_copy_back(const BatchProblem* probs, int nprob, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_copy_back, dim3(1024, nprob), dim3(256), 0, st, probs);
  return hipGetLastError();
}

int cec3d_batch_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cec3d_batch<true>, kT4, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

hipError_t launch_cec3d_seg(bool even, const Geo& g, const float* phi, const float* u, float* out,
                            int* flag, hipStream_t st, Cec3dLaunch lc) {
  const size_t n = (size_t)g.ncells;
  const int ychunk = lc.ychunk > 0 ? lc.ychunk : cec3d_default_ychunk(g);
  dim3 grid((g.nx + 63) / 64, (g.nz + 15) / 16, (g.ny + ychunk - 1) / ychunk);
  if (even)
    hipLaunchKernelGGL(k_cec3d_seg<true>, grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, ychunk, lc.swizzle, flag);
  else
    hipLaunchKernelGGL(k_cec3d_seg<false>, grid, dim3(kThreads), 0, st, phi, u, u + n, u + 2 * n,
                       out, g, ychunk, lc.swizzle, flag);
  return hipGetLastError();
}

// 64 planes per workgroup unless that leaves fewer than 1024 workgroups
// (four per CU), then 32.
int cec3d_default_ychunk(const Geo& g) {
  const long long tiles = (long long)((g.nx + 63) / 64) * ((g.nz + 15) / 16);
  return tiles * ((g.ny + 63) / 64) >= 1024 ? 64 : 32;
}

hipError_t launch_cec3d_multi(int k, bool even, const Geo& g, const float* const* in,
                              float* const* out, const float* u, int* flag, hipStream_t st,
                              int chunk) {
  MfFields fl = {};
  for (int f = 0; f < k && f < kMfMax; ++f) {
    fl.in[f] = in[f];
    fl.out[f] = out[f];
  }
  switch (k) {
    case 1: return launch_cec3d(5, even, g, in[0], u, out[0], flag, st);
    case 2: return launch_mf_k<2>(even, g, fl, u, flag, st, chunk);
    case 4: return launch_mf_k<4>(even, g, fl, u, flag, st, chunk);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cec3d(int variant, bool even, const Geo& g, const float* phi, const float* u,
                        float* out, int* flag, hipStream_t st, Cec3dLaunch lc) {
  if (variant == 1) return launch_cec3d_seg(even, g, phi, u, out, flag, st, lc);
  if (variant == 4) return launch_cec3d_wm<4>(even, g, phi, u, out, flag, st, lc);
  if (variant == 6) return launch_cec3d_wm<8>(even, g, phi, u, out, flag, st, lc);
  if (variant == 7) return launch_cec3d_wl(even, g, phi, u, out, flag, st, lc);
  if (variant == 8) return launch_cec3d_wp(even, g, phi, u, out, flag, st, lc);
  if (variant == 9) return launch_cec3d_wp(even, g, phi, u, out, flag, st, lc, 2);
  if (variant >= 10 && variant <= 13)
    return launch_cec3d_wp(even, g, phi, u, out, flag, st, lc, 1 + (variant & 1), variant < 12 ? 1 : 2);
  if (variant == 14)  // an odd nx has no two-node layout: variant 8 there
    return g.nx % 2 ? launch_cec3d_wp(even, g, phi, u, out, flag, st, lc)
                    : launch_cec3d_wq(even, g, phi, u, out, flag, st, lc);
  if (variant == 5) {
    // the fastest implementation of each parity as measured from 256^3 to
    // 1024^3 (the tuner, sla_tune, measures the grid at hand instead): from
    // 2^24 cells on with an even nx, the march on aligned two-node windows;
    // below, register segments for even steps and the 4-row window march
    // for odd ones; above with an odd nx, the shared-halo march with 16-row
    // groups of 12 waves and 64-plane chunks when 3 divides the window
    // count, with 2-window groups when 2 does, else the 8-row window march,
    // except on odd steps whose 8-row launch would not fill the chip (see
    // wm8_fills)
    if (g.ncells >= (1 << 24) && g.nx % 2 == 0)
      return launch_cec3d_wq(even, g, phi, u, out, flag, st, lc);
    if (g.ncells <= (1 << 24)) {
      if (!even) return launch_cec3d_wm<4>(false, g, phi, u, out, flag, st, lc);
      Cec3dLaunch l = lc;
      if (l.ychunk <= 0) l.ychunk = g.ny >= 512 ? 128 : cec3d_default_ychunk(g);
      return launch_cec3d_seg(true, g, phi, u, out, flag, st, l);
    }
    if (wl_windows(g) == 3) {
      Cec3dLaunch l = lc;
      if (l.ychunk == 0) l.ychunk = -64;
      return launch_cec3d_wp(even, g, phi, u, out, flag, st, l);
    }
    if (wl_windows(g) > 0) return launch_cec3d_wl(even, g, phi, u, out, flag, st, lc);
    if (!even && !wm8_fills(wm_shape(false, g, 8).waves(64)))
      return launch_cec3d_wm<4>(false, g, phi, u, out, flag, st, lc);
    return launch_cec3d_wm<8>(even, g, phi, u, out, flag, st, lc);
  }
  if (variant == 2) return launch_cec3d_v4(even, g, phi, u, out, flag, st, lc);
  return hipErrorInvalidValue;
}

}  // namespace sla
