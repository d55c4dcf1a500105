// Unsplit FEC and BEC steps in one pass over HBM (reach 1).
//
// FEC (eq. intro:FEC):  Phi1 = L_U Phi,  out = Phi1 + (Phi - L_{-U} Phi1)/2.
// BEC (eq. intro:BEC):  Phi1 = L_U Phi,  psi = Phi + (Phi - L_{-U} Phi1)/2,
//                       out = L_U psi.
// Every call is the multilinear interpolation of eq. CIR2D (nested lerps
// x -> y -> z) at the departure point of the node, taken from the node's own
// velocity (the reverse call with the velocity negated).  At reach 1 (every
// |c| < 1) a call reads the 2x2x2 block of nodes between the node and its
// departure point, so stage j of a step needs stage j-1 one node around it.
//
// Layout of the work.  A workgroup owns WX windows of 64 consecutive x (one
// node per lane; 64 - 2K of them are outputs, K = 2 calls for FEC, 3 for
// BEC) by S = 16 rows of y, and marches along z through a chunk of planes.
// Every stage's field lives in LDS for the planes still needed (rings of
// planes); a stage at iteration t works on the plane two behind the plane
// its input stage worked on, so all it reads was written in earlier
// iterations and one barrier per plane suffices.  Stage 0 is the field
// itself, loaded once (plus the K halo rows on each side); the velocity of a
// stage's nodes is read where the stage runs (its second and later reads
// come from L2).  Each node goes through the same FP32 operations, in the
// same order, as the one-call-per-kernel gather chain: the same bits.

#include <type_traits>

#include "common.h"

namespace sla {
namespace {

__device__ __forceinline__ float lerp(float p, float q, float f) { return fmaf(f, q - p, p); }
__device__ __forceinline__ int wrapk(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Buffer access at a per-lane byte offset voff from the row or plane that
// starts soff bytes into the field (soff the same for the whole wave): the
// descriptor is rebased there and has the largest size a descriptor holds,
// so voff alone is range-checked (fields of at most 2^30 cells).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc based_rsrc(const float* field, unsigned soff) {
  const size_t off = unsigned(__builtin_amdgcn_readfirstlane(int(soff)));
  const char* b = reinterpret_cast<const char*>(field) + off;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), short(0), int(0xFFFFFFFFu), 0x00020000);
}
__device__ __forceinline__ float ld_vs(const float* field, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(based_rsrc(field, soff), voff, 0, 0));
}
__device__ __forceinline__ void st_vs(float* field, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), based_rsrc(field, soff), voff,
                                        0, 0);
}

// Workgroups are handed to the 8 XCDs round robin; XCD k takes a contiguous
// range of the tile space instead (x fastest), so neighbouring tiles share
// an L2.
__device__ __forceinline__ int xcd_block() {
  const unsigned n = gridDim.x, L = blockIdx.x;
  const unsigned xcd = L % 8u, q = n / 8u, r = n % 8u;
  return int(xcd * q + min(xcd, r) + L / 8u);
}

template <int SCHEME, int WX_>
struct EcShape {
  static constexpr int K = SCHEME == FEC ? 2 : 3;  // calls per step
  static constexpr int S = 16;                     // output rows per workgroup
  static constexpr int NR = S + 2 * K;             // rows of the field (stage 0)
  static constexpr int WX = WX_;                   // windows per workgroup
  static constexpr int W = 4;                      // waves per window
  static constexpr int USE = 64 - 2 * K;           // outputs per window
  static constexpr int LW = 66;                    // LDS row: lanes + 1 on each side
  static constexpr int PH = 5;                     // planes of the field kept (q-4 .. q)
  static constexpr int RING = 4;                   // planes of a stage kept
  static constexpr int STAGES = SCHEME == FEC ? 1 : 2;  // stages kept in LDS besides the field
};

// One call at a node: the multilinear interpolation of a staged field at the
// departure point for Courant numbers c (already negated for a reverse
// call).  lo / hi: the planes below and above the node's (pm, p0, pp =
// planes p - 1, p, p + 1); r, l: the node's row and LDS column (lane + 1).
template <int LW>
__device__ __forceinline__ float interp(const float* pm, const float* p0, const float* pp, int r, int l,
                                        float cx, float cy, float cz) {
  // s = +1 (c >= 0, -0 included): the far node is at -1 along the axis
  const bool sx = cx >= 0.f, sy = cy >= 0.f, sz = cz >= 0.f;
  const float fx = fabsf(cx), fy = fabsf(cy), fz = fabsf(cz);
  // the 2x2x2 block: lower plane / row / column, then +1
  const float* zl = sz ? pm : p0;
  const float* zh = sz ? p0 : pp;
  const int o = (r - (sy ? 1 : 0)) * LW + (l - (sx ? 1 : 0));
  float v[2][2][2];
  v[0][0][0] = zl[o];
  v[0][0][1] = zl[o + 1];
  v[0][1][0] = zl[o + LW];
  v[0][1][1] = zl[o + LW + 1];
  v[1][0][0] = zh[o];
  v[1][0][1] = zh[o + 1];
  v[1][1][0] = zh[o + LW];
  v[1][1][1] = zh[o + LW + 1];
  // along each axis the anchor (the node's own index) and the far node: for
  // s = +1 the anchor is the upper of the pair.  x first, then y, then z, as
  // in every other interpolation of the library.
  float wx[2][2];
#pragma unroll
  for (int zi = 0; zi < 2; ++zi)
#pragma unroll
    for (int yi = 0; yi < 2; ++yi)
      wx[zi][yi] = lerp(sx ? v[zi][yi][1] : v[zi][yi][0], sx ? v[zi][yi][0] : v[zi][yi][1], fx);
  float wy[2];
#pragma unroll
  for (int zi = 0; zi < 2; ++zi)
    wy[zi] = lerp(sy ? wx[zi][1] : wx[zi][0], sy ? wx[zi][0] : wx[zi][1], fy);
  return lerp(sz ? wy[1] : wy[0], sz ? wy[0] : wy[1], fz);
}

__device__ __forceinline__ bool over1(float c) { return fabsf(c) >= 1.f; }

template <int SCHEME, int WX_>
__global__ __launch_bounds__(256 * WX_, (SCHEME == FEC && WX_ == 1) ? 3 : 2) void k_ec_march(
    const float* __restrict__ phi, const float* __restrict__ ux, const float* __restrict__ uy,
    const float* __restrict__ uz, float* __restrict__ out, Geo g, int chunk, int* flag) {
  using Sh = EcShape<SCHEME, WX_>;
  constexpr int K = Sh::K, S = Sh::S, NR = Sh::NR, WX = Sh::WX, W = Sh::W, LW = Sh::LW;
  constexpr int PH = Sh::PH, RING = Sh::RING;
  // rows per wave: stage j covers rows j .. NR - 1 - j
  constexpr int R0 = (NR + W - 1) / W;
  constexpr int R1 = (NR - 2 + W - 1) / W;
  constexpr int R2 = (NR - 4 + W - 1) / W;
  constexpr int R3 = (NR - 6 + W - 1) / W;
  __shared__ float lphi[PH][WX][NR][LW];
  __shared__ float lst[Sh::STAGES][RING][WX][NR][LW];
  const int lane = threadIdx.x & 63, xi = (threadIdx.x >> 6) % WX, w = (threadIdx.x >> 6) / WX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int nwx = (nx + Sh::USE - 1) / Sh::USE, ngx = (nwx + WX - 1) / WX, ngy = (ny + S - 1) / S;
  const int nch = (nz + chunk - 1) / chunk;
  const int blk = xcd_block();
  if (blk >= ngx * ngy * nch) return;  // the whole workgroup
  const int wx0 = (blk % ngx) * WX, gy = (blk / ngx) % ngy, ch = blk / (ngx * ngy);
  const bool wx_ok = wx0 + xi < nwx;  // the same for the whole wave
  const int wx = min(wx0 + xi, nwx - 1);
  const unsigned vx = 4u * unsigned(wrapk(wx * Sh::USE - K + lane, nx));
  const unsigned rowb = 4u * unsigned(nx);
  const int y0 = gy * S;  // row r of a stage is y0 - K + r
  const int m0 = ch * chunk, m1 = min(m0 + chunk, nz);
  const float lx = g.lam[0], ly = g.lam[1], lz = g.lam[2];
  const int l = lane + 1;  // LDS column
  // the padding columns are read only by lanes whose results are unused
  for (int i = threadIdx.x; i < PH * WX * NR; i += blockDim.x) {
    float* row = &lphi[0][0][0][0] + size_t(i) * LW;
    row[0] = 0.f;
    row[LW - 1] = 0.f;
  }
  for (int i = threadIdx.x; i < Sh::STAGES * RING * WX * NR; i += blockDim.x) {
    float* row = &lst[0][0][0][0][0] + size_t(i) * LW;
    row[0] = 0.f;
    row[LW - 1] = 0.f;
  }
  // Byte offsets within a plane of the rows each stage of this wave handles
  // (stage j: rows j + w Rj + k), computed once: the divisions of the
  // periodic wrap run on the vector unit even for wave-uniform values.
  auto rowoff = [&](int r) { return unsigned(__builtin_amdgcn_readfirstlane(wrapk(y0 - K + r, ny))) * rowb; };
  // A wave's rows past the end of a stage's range repeat the stage's last
  // row: they recompute (and rewrite) the same values, so every row runs
  // the same branch-free code and the rows' LDS reads overlap.
  auto srow = [&](int j, int rj, int k) { return min(j + w * rj + k, NR - 1 - j); };
  unsigned off0[R0], off1[R1], off2[R2], off3[R3];
#pragma unroll
  for (int k = 0; k < R0; ++k) off0[k] = rowoff(srow(0, R0, k));
#pragma unroll
  for (int k = 0; k < R1; ++k) off1[k] = rowoff(srow(1, R1, k));
#pragma unroll
  for (int k = 0; k < R2; ++k) off2[k] = rowoff(srow(2, R2, k));
#pragma unroll
  for (int k = 0; k < R3; ++k) off3[k] = rowoff(srow(3, R3, k));
  // plane of stage j at iteration t: q - 2 j with q = m0 - K + t, wrapped;
  // advanced by one plane per iteration without a division
  const unsigned plb = unsigned(ny) * rowb;
  int pl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) pl[j] = __builtin_amdgcn_readfirstlane(wrapk(m0 - K - 2 * j, nz));
  auto next = [&](int p) { return p + 1 < nz ? p + 1 : 0; };
  // ring slots of a march plane p (p >= m0 - K - 8: offset to stay >= 0)
  auto slot5 = [&](int p) { return (p - m0 + 20) % PH; };
  auto slot4 = [&](int p) { return (p - m0 + 20) & (RING - 1); };

  const int iters = (m1 - m0) + 3 * K;
  bool over = false;
  // prefetch registers: the field rows of stage 0, the velocity of each
  // stage's rows (stage j works on plane q - 2 j at iteration t, q = m0 - K + t)
  float fp[R0];
  float fu1[3][R1], fu2[3][R2], fu3[3][R3];
  // np[j]: the plane of stage j at the iteration being prefetched
  auto prefetch = [&](const int (&np)[4]) {
    const unsigned pq = unsigned(np[0]) * plb;
#pragma unroll
    for (int k = 0; k < R0; ++k) fp[k] = ld_vs(phi, vx, pq + off0[k]);
    const unsigned p1 = unsigned(np[1]) * plb;
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const unsigned o = p1 + off1[k];
      fu1[0][k] = ld_vs(ux, vx, o);
      fu1[1][k] = ld_vs(uy, vx, o);
      fu1[2][k] = ld_vs(uz, vx, o);
    }
    const unsigned p2 = unsigned(np[2]) * plb;
#pragma unroll
    for (int k = 0; k < R2; ++k) {
      const unsigned o = p2 + off2[k];
      fu2[0][k] = ld_vs(ux, vx, o);
      fu2[1][k] = ld_vs(uy, vx, o);
      fu2[2][k] = ld_vs(uz, vx, o);
    }
    if (SCHEME == BEC) {
      const unsigned p3 = unsigned(np[3]) * plb;
#pragma unroll
      for (int k = 0; k < R3; ++k) {
        const unsigned o = p3 + off3[k];
        fu3[0][k] = ld_vs(ux, vx, o);
        fu3[1][k] = ld_vs(uy, vx, o);
        fu3[2][k] = ld_vs(uz, vx, o);
      }
    }
  };
  const bool lane_out = lane >= K && lane < 64 - K && wx * Sh::USE + lane - K < nx;
  if (wx_ok) prefetch(pl);
  for (int t = 0; t < iters; ++t) {
    const int q = m0 - K + t;
    int npl[4];  // the planes of iteration t + 1
#pragma unroll
    for (int j = 0; j < 4; ++j) npl[j] = next(pl[j]);
    __syncthreads();  // the writes of earlier iterations are visible, their reads done
    if (wx_ok) {
      // stage 0: the field of plane q
#pragma unroll
      for (int k = 0; k < R0; ++k) lphi[slot5(q)][xi][srow(0, R0, k)][l] = fp[k];
      float u1[3][R1], u2[3][R2], u3[3][R3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < R1; ++k) u1[d][k] = fu1[d][k];
#pragma unroll
        for (int k = 0; k < R2; ++k) u2[d][k] = fu2[d][k];
        if (SCHEME == BEC)
#pragma unroll
          for (int k = 0; k < R3; ++k) u3[d][k] = fu3[d][k];
      }
      if (t + 1 < iters) prefetch(npl);
      // stage 1 at plane q - 2: Phi1 = L_U Phi
      {
        const int p = q - 2;
        const float* pm = &lphi[slot5(p - 1)][xi][0][0];
        const float* p0 = &lphi[slot5(p)][xi][0][0];
        const float* pp = &lphi[slot5(p + 1)][xi][0][0];
#pragma unroll
        for (int k = 0; k < R1; ++k) {
          const int r = srow(1, R1, k);
          const float cx = u1[0][k] * lx, cy = u1[1][k] * ly, cz = u1[2][k] * lz;
          over |= over1(cx) || over1(cy) || over1(cz);
          lst[0][slot4(p)][xi][r][l] = interp<LW>(pm, p0, pp, r, l, cx, cy, cz);
        }
      }
      // stage 2 at plane q - 4: the reverse call on Phi1, then FEC's result
      // or BEC's psi
      {
        const int p = q - 4;
        const float* pm = &lst[0][slot4(p - 1)][xi][0][0];
        const float* p0 = &lst[0][slot4(p)][xi][0][0];
        const float* pp = &lst[0][slot4(p + 1)][xi][0][0];
        const float* f0 = &lphi[slot5(p)][xi][0][0];
        const unsigned po = unsigned(pl[2]) * plb;
#pragma unroll
        for (int k = 0; k < R2; ++k) {
          const int r = srow(2, R2, k);
          const float cx = -(u2[0][k] * lx), cy = -(u2[1][k] * ly), cz = -(u2[2][k] * lz);
          const float rv = interp<LW>(pm, p0, pp, r, l, cx, cy, cz);
          const float fv = f0[r * LW + l];
          if (SCHEME == FEC) {
            // out = Phi1 + (Phi - L_{-U} Phi1)/2
            const float o = fmaf(0.5f, fv - rv, p0[r * LW + l]);
            if (t >= 3 * K && lane_out && y0 - K + r < ny) st_vs(out, vx, po + off2[k], o);
          } else {
            lst[Sh::STAGES - 1][slot4(p)][xi][r][l] = fmaf(0.5f, fv - rv, fv);  // psi
          }
        }
      }
      // stage 3 (BEC) at plane q - 6: out = L_U psi
      if (SCHEME == BEC) {
        const int p = q - 6;
        const float* pm = &lst[Sh::STAGES - 1][slot4(p - 1)][xi][0][0];
        const float* p0 = &lst[Sh::STAGES - 1][slot4(p)][xi][0][0];
        const float* pp = &lst[Sh::STAGES - 1][slot4(p + 1)][xi][0][0];
        const unsigned po = unsigned(pl[3]) * plb;
#pragma unroll
        for (int k = 0; k < R3; ++k) {
          const int r = srow(3, R3, k);
          const float cx = u3[0][k] * lx, cy = u3[1][k] * ly, cz = u3[2][k] * lz;
          const float o = interp<LW>(pm, p0, pp, r, l, cx, cy, cz);
          if (t >= 3 * K && lane_out && y0 - K + r < ny) st_vs(out, vx, po + off3[k], o);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) pl[j] = npl[j];
  }
  if (over) *flag = 1;
}

}  // namespace

// Reach-1 unsplit FEC or BEC step of a 3D grid of at most 2^30 cells (ny >=
// 2 at 2^30), all calls in one kernel.
hipError_t launch_ec_march(int scheme, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  auto shape = [&](auto sch) {
    constexpr int SC = decltype(sch)::value;
    using Sh = EcShape<SC, 1>;
    const long long groups =
        (long long)(((g.nx + Sh::USE - 1) / Sh::USE + Sh::WX - 1) / Sh::WX) * ((g.ny + Sh::S - 1) / Sh::S);
    // march chunks of 128 planes, shorter while that leaves under 1024 workgroups
    int chunk = 128;
    while (chunk > 16 && groups * ((g.nz + chunk - 1) / chunk) < 1024) chunk /= 2;
    const dim3 grid(unsigned(groups * ((g.nz + chunk - 1) / chunk)));
    hipLaunchKernelGGL((k_ec_march<SC, 1>), grid, dim3(64 * Sh::W * Sh::WX), 0, st, phi, u, u + n,
                       u + 2 * n, out, g, chunk, flag);
    return hipGetLastError();
  };
  if (scheme == FEC) return shape(std::integral_constant<int, FEC>{});
  if (scheme == BEC) return shape(std::integral_constant<int, BEC>{});
  return hipErrorInvalidValue;
}

}  // namespace sla
