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
// itself, loaded once (plus the K halo rows on each side); the velocity of
// a node is loaded once, for stage 1, and kept in registers for the node's
// later stages, which reach it two and four iterations later (a ring of
// register sets).  Each node goes through the same FP32 operations, in the
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

// Buffer access within one plane of a field: the descriptor is rebased on
// the plane (once per plane and field) and has the largest size a
// descriptor holds; an access adds the row's byte offset within the plane
// (the same for the whole wave, a scalar operand) and the lane's offset
// within the row.  Planes of fields of at most 2^30 cells with nz >= 2 are
// under 2^31 bytes, so every offset fits.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc plane_rsrc(const float* field, unsigned plane_off) {
  const size_t off = unsigned(__builtin_amdgcn_readfirstlane(int(plane_off)));
  const char* b = reinterpret_cast<const char*>(field) + off;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), short(0), int(0xFFFFFFFFu), 0x00020000);
}
__device__ __forceinline__ float ld_row(Rsrc r, unsigned lane_off, unsigned row_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, lane_off, row_off, 0));
}
__device__ __forceinline__ void st_row(Rsrc r, unsigned lane_off, unsigned row_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, lane_off, row_off, 0);
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
// call).  Along each axis the anchor is the node's own index and the far
// node lies one step against the sign of c (c >= 0, -0 included: index - 1,
// else index + 1), so the eight values are read at the node and at its far
// neighbours, each at its own per-lane address, and enter the lerps without
// any selection.  A call is split into its reads (corners) and its
// arithmetic (blend) so that a wave issues the reads of all its nodes
// before the first result is needed.
struct Call {
  float v[8];  // own plane: node, far x, far y, far xy; then the far plane
  float fx, fy, fz;
};
// na: the node in its own plane; nf: the same row and column in the far plane
template <int LW>
__device__ __forceinline__ void corners(Call& k, const float* na, const float* nf, float cx, float cy,
                                        float cz) {
  const int dx = cx >= 0.f ? -1 : 1;
  const int dy = cy >= 0.f ? -LW : LW;
  k.fx = fabsf(cx);
  k.fy = fabsf(cy);
  k.fz = fabsf(cz);
  k.v[0] = na[0];
  k.v[1] = na[dx];
  k.v[2] = na[dy];
  k.v[3] = na[dy + dx];
  k.v[4] = nf[0];
  k.v[5] = nf[dx];
  k.v[6] = nf[dy];
  k.v[7] = nf[dy + dx];
}
// x first, then y, then z, as in every other interpolation of the library
__device__ __forceinline__ float blend(const Call& k) {
  const float a = lerp(lerp(k.v[0], k.v[1], k.fx), lerp(k.v[2], k.v[3], k.fx), k.fy);
  const float f = lerp(lerp(k.v[4], k.v[5], k.fx), lerp(k.v[6], k.v[7], k.fx), k.fy);
  return lerp(a, f, k.fz);
}

// True if a Courant number of the node is beyond reach 1 (NaN is not).
__device__ __forceinline__ bool over3(float cx, float cy, float cz) {
  return fmaxf(fmaxf(fabsf(cx), fabsf(cy)), fabsf(cz)) >= 1.f;
}

template <int SCHEME, int WX_>
__global__ __launch_bounds__(256 * WX_, (SCHEME == FEC && WX_ == 1) ? 3 : 2) void k_ec_march(
    const float* __restrict__ phi, const float* __restrict__ ux, const float* __restrict__ uy,
    const float* __restrict__ uz, float* __restrict__ out, Geo g, int span, int* flag) {
  using Sh = EcShape<SCHEME, WX_>;
  constexpr int K = Sh::K, S = Sh::S, NR = Sh::NR, WX = Sh::WX, W = Sh::W, LW = Sh::LW;
  constexpr int PH = Sh::PH, RING = Sh::RING;
  // Rows per wave: stage j covers rows j .. NR - 1 - j.  A wave keeps the
  // velocity it loaded for its stage-1 rows for its later stages (two and
  // four iterations later) in a ring of register sets, so each node's
  // velocity is read once.  FEC: a wave's stage-1 rows are 1 + R2 w ..
  // 2 + R2 w + R2, its stage-2 rows and one on each side (neighbouring waves
  // overlap by two rows, computed twice).  BEC: every stage of a wave works
  // on the same RU rows 1 + RU w .., each stage writing only those in its
  // own range.
  constexpr bool VRING = SCHEME == FEC && (NR - 4) % W == 0;
  constexpr bool URING = SCHEME == BEC && (NR - 2) % W == 0;
  constexpr int RU = (NR - 2 + W - 1) / W;
  constexpr int R0 = (NR + W - 1) / W;
  constexpr int R2 = URING ? RU : (NR - 4 + W - 1) / W;
  constexpr int R3 = URING ? RU : (NR - 6 + W - 1) / W;
  constexpr int R1 = VRING ? R2 + 2 : RU;
  constexpr int NSET = VRING ? 4 : URING ? 6 : 2;  // velocity register sets
  __shared__ float lphi[PH][WX][NR][LW];
  __shared__ float lst[Sh::STAGES][RING][WX][NR][LW];
  // the wave's window and row group, the same for all its lanes (made
  // scalar so that row addresses are a scalar plus the lane's column)
  const int lane = threadIdx.x & 63;
  const int xi = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) % WX);
  const int w = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) / WX);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int nwx = (nx + Sh::USE - 1) / Sh::USE, ngx = (nwx + WX - 1) / WX, ngy = (ny + S - 1) / S;
  const long long total = (long long)ngx * ngy * nz;  // the line of (group, plane) pairs
  const int blk = xcd_block();
  long long i0, i1;
  if (span > 0) {  // a range of the line: persistent workgroups
    i0 = (long long)blk * span;
    i1 = min(i0 + (long long)span, total);
  } else {  // one chunk of -span planes of one group, groups fastest
    const int ng = ngx * ngy, ch = blk / ng, grp = blk - ch * ng;
    i0 = (long long)grp * nz + (long long)ch * -span;
    i1 = (long long)grp * nz + min(nz, (ch + 1) * -span);
  }
  const float lx = g.lam[0], ly = g.lam[1], lz = g.lam[2];
  const unsigned rowb = 4u * unsigned(nx);
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
  bool over = false;
  // one run: planes m0 .. m1 - 1 of one group (the same for the whole
  // workgroup); a run restarts the stage pipeline
  while (i0 < i1) {
    const int grp = int(i0 / nz), m0 = int(i0 - (long long)grp * nz);
    const int m1 = int(min((long long)nz, (long long)m0 + (i1 - i0)));
    i0 += m1 - m0;
    const int wx0 = (grp % ngx) * WX, gy = grp / ngx;
    const bool wx_ok = wx0 + xi < nwx;  // the same for the whole wave
    const int wx = min(wx0 + xi, nwx - 1);
    const unsigned vx = 4u * unsigned(wrapk(wx * Sh::USE - K + lane, nx));
    const int y0 = gy * S;  // row r of a stage is y0 - K + r
    // Byte offsets within a plane of the rows each stage of this wave handles
    // (stage j: rows j + w Rj + k), computed once: the divisions of the
    // periodic wrap run on the vector unit even for wave-uniform values.
    auto rowoff = [&](int r) { return unsigned(__builtin_amdgcn_readfirstlane(wrapk(y0 - K + r, ny))) * rowb; };
    // A wave's rows past the end of a stage's range repeat the stage's last
    // row: they recompute (and rewrite) the same values, so every row runs
    // the same branch-free code and the rows' LDS reads overlap.
    auto srow = [&](int j, int rj, int k) {
      if (URING && j >= 1) return 1 + RU * w + k;
      return min(j + w * (VRING && j == 1 ? R2 : rj) + k, NR - 1 - j);
    };
    // a row of stage j that the stage writes (URING: all rows are computed)
    auto mine = [&](int j, int r) { return !URING || (r >= j && r <= NR - 1 - j); };
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
    // prefetch registers: the field rows of stage 0 (written to LDS at the
    // start of the next iteration), and two sets of the velocity of each
    // stage's rows, the one in use and the one loading (stage j works on
    // plane q - 2 j at iteration t, q = m0 - K + t)
    float fp[R0];
    constexpr bool RINGED = VRING || URING;
    float fu1[NSET][3][R1], fu2[RINGED ? 1 : 2][3][R2], fu3[RINGED ? 1 : 2][3][R3];
    if (RINGED) {  // sets read (by later stages) before any load reached them
#pragma unroll
      for (int b = 0; b < NSET; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int k = 0; k < R1; ++k) fu1[b][d][k] = 0.f;
    }
    // np[j]: the plane of stage j at the iteration being prefetched
    auto prefetch = [&](auto setc, const int (&np)[4]) {
      constexpr int B = decltype(setc)::value;
      const Rsrc rp = plane_rsrc(phi, unsigned(np[0]) * plb);
#pragma unroll
      for (int k = 0; k < R0; ++k) fp[k] = ld_row(rp, vx, off0[k]);
      {
        const unsigned o = unsigned(np[1]) * plb;
        const Rsrc rx = plane_rsrc(ux, o), ry = plane_rsrc(uy, o), rz = plane_rsrc(uz, o);
#pragma unroll
        for (int k = 0; k < R1; ++k) {
          fu1[B][0][k] = ld_row(rx, vx, off1[k]);
          fu1[B][1][k] = ld_row(ry, vx, off1[k]);
          fu1[B][2][k] = ld_row(rz, vx, off1[k]);
        }
      }
      if (!RINGED) {
        const unsigned o = unsigned(np[2]) * plb;
        const Rsrc rx = plane_rsrc(ux, o), ry = plane_rsrc(uy, o), rz = plane_rsrc(uz, o);
#pragma unroll
        for (int k = 0; k < R2; ++k) {
          fu2[B][0][k] = ld_row(rx, vx, off2[k]);
          fu2[B][1][k] = ld_row(ry, vx, off2[k]);
          fu2[B][2][k] = ld_row(rz, vx, off2[k]);
        }
      }
      if (SCHEME == BEC && !RINGED) {
        const unsigned o = unsigned(np[3]) * plb;
        const Rsrc rx = plane_rsrc(ux, o), ry = plane_rsrc(uy, o), rz = plane_rsrc(uz, o);
#pragma unroll
        for (int k = 0; k < R3; ++k) {
          fu3[B][0][k] = ld_row(rx, vx, off3[k]);
          fu3[B][1][k] = ld_row(ry, vx, off3[k]);
          fu3[B][2][k] = ld_row(rz, vx, off3[k]);
        }
      }
    };
    const bool lane_out = lane >= K && lane < 64 - K && wx * Sh::USE + lane - K < nx;
    // column l of row 0 of a plane of a stage's ring
    auto col = [&](float* plane) { return plane + l; };
    // Far plane of a node (below if its z Courant number is >= 0, else
    // above) as an element offset from its own plane, from the ring slots of
    // the three planes: a per-lane choice between two scalars, kept opaque so
    // that the compiler selects the offsets rather than recomputing ring slots
    // per lane.
    constexpr int PS = WX * NR * LW;  // elements per ring plane
    auto far_off = [&](int own, int below, int above, float cz) {
      int dm = (below - own) * PS, dp = (above - own) * PS;
      asm("" : "+s"(dm), "+s"(dp));  // no instruction: hides the products from the select
      return cz >= 0.f ? dm : dp;
    };
    auto body = [&](auto setc, int t) {
      constexpr int B = decltype(setc)::value;
      const int q = m0 - K + t;
      int npl[4];  // the planes of iteration t + 1
#pragma unroll
      for (int j = 0; j < 4; ++j) npl[j] = next(pl[j]);
      __syncthreads();  // the writes of earlier iterations are visible, their reads done
      if (wx_ok) {
        // stage 0: the field of plane q
#pragma unroll
        for (int k = 0; k < R0; ++k) lphi[slot5(q)][xi][srow(0, R0, k)][l] = fp[k];
      // unconditional: past the run's end it reads valid planes whose values
      // go unused (a conditional load would merge old and new register values
      // and make the wave wait for the loads it has just issued)
      prefetch(std::integral_constant<int, (B + 1) % NSET>{}, npl);
        // Stage j reads planes written in earlier iterations only (its input
        // stage ran two planes ahead) and writes other ring slots, so the
        // stages of one iteration are independent: each issues the reads of
        // all its rows before its first result, the last stage first.
        const int p1 = q - 2, p2 = q - 4, p3 = q - 6;
        // stage 3 (BEC) at plane q - 6: out = L_U psi
        if (SCHEME == BEC) {
          const float* a0 = col(&lst[Sh::STAGES - 1][slot4(p3)][xi][0][0]);
          Call c[R3];
#pragma unroll
          for (int k = 0; k < R3; ++k) {
            const int r = srow(3, R3, k);
            constexpr int B3 = (B + NSET - 4) % NSET;  // the ring set of four iterations ago
            const float cx = (URING ? fu1[B3][0][k] : fu3[RINGED ? 0 : B][0][k]) * lx;
            const float cy = (URING ? fu1[B3][1][k] : fu3[RINGED ? 0 : B][1][k]) * ly;
            const float cz = (URING ? fu1[B3][2][k] : fu3[RINGED ? 0 : B][2][k]) * lz;
            const float* na = a0 + r * LW;
            corners<LW>(c[k], na, na + far_off(slot4(p3), slot4(p3 - 1), slot4(p3 + 1), cz), cx, cy, cz);
          }
          const Rsrc ro = plane_rsrc(out, unsigned(pl[3]) * plb);
#pragma unroll
          for (int k = 0; k < R3; ++k) {
            const float o = blend(c[k]);
            const int r = srow(3, R3, k);
            if (t >= 3 * K && lane_out && y0 - K + r < ny && mine(3, r)) st_row(ro, vx, off3[k], o);
          }
        }
        // stage 2 at plane q - 4: the reverse call on Phi1, then FEC's result
        // or BEC's psi
        {
          const float* a0 = col(&lst[0][slot4(p2)][xi][0][0]);
          const float* f0 = col(&lphi[slot5(p2)][xi][0][0]);
          Call c[R2];
          float fv[R2];
#pragma unroll
          for (int k = 0; k < R2; ++k) {
            const int r = srow(2, R2, k);
            // the velocity of row r: FEC's ring set of two iterations ago
            // (stage 1 then worked on this plane; row r is its row k + 1)
            constexpr int B2 = (B + NSET - 2) % NSET;
            constexpr int K1 = VRING ? 1 : 0;  // FEC: row r is stage 1's row k + 1
            const float vx_ = RINGED ? fu1[B2][0][k + K1] : fu2[RINGED ? 0 : B][0][k];
            const float vy_ = RINGED ? fu1[B2][1][k + K1] : fu2[RINGED ? 0 : B][1][k];
            const float vz_ = RINGED ? fu1[B2][2][k + K1] : fu2[RINGED ? 0 : B][2][k];
            const float cx = -(vx_ * lx), cy = -(vy_ * ly), cz = -(vz_ * lz);
            const float* na = a0 + r * LW;
            corners<LW>(c[k], na, na + far_off(slot4(p2), slot4(p2 - 1), slot4(p2 + 1), cz), cx, cy, cz);
            fv[k] = f0[r * LW];
          }
          const Rsrc ro = plane_rsrc(out, unsigned(pl[2]) * plb);
#pragma unroll
          for (int k = 0; k < R2; ++k) {
            const int r = srow(2, R2, k);
            const float rv = blend(c[k]);
            if (SCHEME == FEC) {
              // out = Phi1 + (Phi - L_{-U} Phi1)/2, Phi1 at the node being the
              // reverse call's anchor
              const float o = fmaf(0.5f, fv[k] - rv, c[k].v[0]);
              if (t >= 3 * K && lane_out && y0 - K + r < ny) st_row(ro, vx, off2[k], o);
            } else {
              if (mine(2, r)) lst[Sh::STAGES - 1][slot4(p2)][xi][r][l] = fmaf(0.5f, fv[k] - rv, fv[k]);  // psi
            }
          }
        }
        // stage 1 at plane q - 2: Phi1 = L_U Phi; every node of the later
        // stages is a node of this one, with the same velocity: the reach is
        // checked here
        {
          const float* a0 = col(&lphi[slot5(p1)][xi][0][0]);
          Call c[R1];
#pragma unroll
          for (int k = 0; k < R1; ++k) {
            const int r = srow(1, R1, k);
            const float cx = fu1[B][0][k] * lx, cy = fu1[B][1][k] * ly, cz = fu1[B][2][k] * lz;
            over |= over3(cx, cy, cz);
            const float* na = a0 + r * LW;
            corners<LW>(c[k], na, na + far_off(slot5(p1), slot5(p1 - 1), slot5(p1 + 1), cz), cx, cy, cz);
          }
#pragma unroll
          for (int k = 0; k < R1; ++k) lst[0][slot4(p1)][xi][srow(1, R1, k)][l] = blend(c[k]);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) pl[j] = npl[j];
    };
    if (wx_ok) prefetch(std::integral_constant<int, 0>{}, pl);
    for (int t = 0; t < iters; t += NSET) {
      body(std::integral_constant<int, 0>{}, t);
      if (t + 1 < iters) body(std::integral_constant<int, 1>{}, t + 1);
      if (NSET >= 4) {
        if (t + 2 < iters) body(std::integral_constant<int, 2 % NSET>{}, t + 2);
        if (t + 3 < iters) body(std::integral_constant<int, 3 % NSET>{}, t + 3);
      }
      if (NSET == 6) {
        if (t + 4 < iters) body(std::integral_constant<int, 4 % NSET>{}, t + 4);
        if (t + 5 < iters) body(std::integral_constant<int, 5 % NSET>{}, t + 5);
      }
    }
  }
  if (over) *flag = 1;
}

}  // namespace

// Reach-1 unsplit FEC or BEC step of a 3D grid of at most 2^30 cells (ny >=
// 2 at 2^30), all calls in one kernel.
hipError_t launch_ec_march(int scheme, const Geo& g, const float* phi, const float* u, float* out,
                           int* flag, hipStream_t st, int shape) {
  const size_t n = (size_t)g.ncells;
  auto go = [&](auto sch) {
    constexpr int SC = decltype(sch)::value;
    using Sh = EcShape<SC, 1>;
    auto kern = k_ec_march<SC, 1>;
    const long long groups =
        (long long)(((g.nx + Sh::USE - 1) / Sh::USE + Sh::WX - 1) / Sh::WX) * ((g.ny + Sh::S - 1) / Sh::S);
    const long long total = groups * g.nz;
    static int cus = 0, fit = 0;
    if (!cus) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, kern, 64 * Sh::W * Sh::WX, 0) != hipSuccess ||
          fit < 1)
        fit = 1;
    }
    long long blocks;
    int span;
    if (shape == 0) {
      // March chunks (faster than persistent ranges: the workgroups in
      // flight then march the same planes of neighbouring groups, whose
      // shared halo rows meet in L2).  The chunk count minimises the time
      // model rounds x (planes per chunk + pipeline fill), rounds being the
      // waves of workgroups the chip holds at once; chunks of 16 planes or
      // more.
      const long long slots = (long long)cus * fit;
      long long best = -1;
      for (int nch = 1; nch == 1 || (g.nz + nch - 1) / nch >= 16; ++nch) {
        const long long rounds = (groups * nch + slots - 1) / slots;
        const long long cost = rounds * ((g.nz + nch - 1) / nch + 3 * Sh::K);
        if (best < 0 || cost < best) {
          best = cost;
          shape = -((g.nz + nch - 1) / nch);
        }
      }
    }
    if (shape < 0) {  // chunks of -shape planes, one workgroup each
      span = shape;
      blocks = groups * ((g.nz - shape - 1) / -shape);
    } else {  // persistent: shape workgroups per CU (at most as many as fit), each a range of the line
      blocks = (long long)cus * min(shape, fit);
      blocks = max(1LL, min(blocks, total / 16));  // at least 16 planes each
      span = int((total + blocks - 1) / blocks);
      blocks = (total + span - 1) / span;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * Sh::W * Sh::WX), 0, st, phi, u, u + n,
                       u + 2 * n, out, g, span, flag);
    return hipGetLastError();
  };
  if (scheme == FEC) return go(std::integral_constant<int, FEC>{});
  if (scheme == BEC) return go(std::integral_constant<int, BEC>{});
  return hipErrorInvalidValue;
}

}  // namespace sla
