// Advection kernels for gfx950: CIR, fused unsplit FEC/BEC, and the per-axis
// third-order sweep.
//
// Every kernel decomposes the Courant number of a node the same way
// (section 3 of the paper defines s_i = sgn(u_i) and U_i = |u_i| dt/dx; at
// CFL > 1 the stencil moves with the departure point, section 4):
//   c = u * fl32(dt/dx)          one FP32 multiply
//   n = floor(|c|), f = |c| - n  (f exact in FP32)
//   anchor offset oa = -s n, far offset ob = -s (n + 1), s = +1 if c >= 0
// Offsets stay integers, so a departure point is never formed as an FP32
// coordinate and index arithmetic stays exact on any grid size.
// Interpolation is p + f (q - p) with p the anchor: integer Courant numbers
// and constant fields come out bit-exact.

#include <algorithm>
#include <utility>

#include "common.h"

#include "../../include/sla.h"

namespace sla {
namespace {

constexpr int kThreads = 256;

struct Dep {
  int oa;  // anchor offset, cells
  int ob;  // far offset, cells
  float f; // fraction in [0, 1)
};

// Departure of a node with Courant number c, for kernels whose halo serves a
// reach of R cells.  A Courant number needing more is clamped to the reach
// (every access stays in bounds) and recorded in *flag.
template <int R>
__device__ __forceinline__ Dep depart(float c, int* flag) {
  const float mag = fabsf(c);
  float nf = floorf(mag);
  const float f = mag - nf;
  if (!(nf <= float(R - 1))) {
    if (nf == nf) *flag = 1;  // NaN is not an overflow: it propagates as NaN
    nf = float(R - 1);
  }
  const int n = int(nf);
  const bool pos = c >= 0.f;  // -0.0 counts as positive
  Dep d;
  d.oa = pos ? -n : n;
  d.ob = pos ? -(n + 1) : (n + 1);
  d.f = f;
  return d;
}
// The same decomposition and clamp with the overflow or-ed into `over`, for
// kernels that store the flag once instead of a conditional store per call.
template <int R>
__device__ __forceinline__ Dep depart_o(float c, bool& over) {
  const float mag = fabsf(c);
  const float nf = floorf(mag);
  const float f = mag - nf;
  over |= nf > float(R - 1);  // false for NaN, which propagates
  const int n = int(fminf(nf, float(R - 1)));
  const bool pos = c >= 0.f;  // -0.0 counts as positive
  Dep d;
  d.oa = pos ? -n : n;
  d.ob = pos ? -(n + 1) : (n + 1);
  d.f = f;
  return d;
}

__device__ __forceinline__ float lerp(float p, float q, float f) { return fmaf(f, q - p, p); }

// v within one period of [0, n)
__device__ __forceinline__ int wrap1(int v, int n) {
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}
// any v (used where a halo may exceed a short axis)
__device__ __forceinline__ int wrapk(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

// Run f(i) for i = start + STRIDE k < N, unrolled to a compile-time trip
// count so that a thread's independent LDS reads are all issued before the
// first result is needed.
template <int N, int STRIDE, typename F>
__device__ __forceinline__ void for_strided(int start, F&& f) {
#pragma unroll
  for (int k = 0; k < (N + STRIDE - 1) / STRIDE; ++k) {
    const int i = start + k * STRIDE;
    if (i < N) f(i);
  }
}

// ---------------------------------------------------------------------------
// One interpolation call per node, gathered from global memory (served by
// L1/L2), CPT nodes per thread: the CPT rows y0 + 4j + threadIdx.y of a
// 64-wide x window, so a thread issues all its velocity loads, then all its
// gathers, before it needs the first of them.  MODE 0, CIR: out = L_U[a]
// (section 3 first equation; eq. CIR2D; the same tensor product in 3D).
// The chained unsplit FEC / BEC use the reverse call: MODE 1, FEC's last
// call: out = a + (b - L_{-U}[a])/2 with a = Phi1 and b = Phi; MODE 2, BEC's
// middle call: out = b + (b - L_{-U}[a])/2 (psi).  out may be b: a thread
// reads b only at its own nodes, before it writes there.  Interpolation
// order x, then y, then z, as in every kernel here: FEC = MODE 0, MODE 1;
// BEC = MODE 0, MODE 2, MODE 0 give the fused k_ec's results bit for bit.
// ---------------------------------------------------------------------------
template <int NDIM, int MODE, int CPT>
__global__ __launch_bounds__(kThreads) void k_gather(const float* __restrict__ a, const float* b,
                                                     const float* __restrict__ ux,
                                                     const float* __restrict__ uy,
                                                     const float* __restrict__ uz, float* out,
                                                     Geo g, int* flag) {
  constexpr int R = SLA_MAX_REACH;
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int z = blockIdx.z;
  if (x >= g.nx) return;
  const int plane = g.nx * g.ny;
  const float sgn = MODE == 0 ? 1.f : -1.f;  // MODE 1, 2: the reverse call
  int idx[CPT];
  Dep dx[CPT], dy[CPT], dz[CPT];
  bool ok[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int y = blockIdx.y * (4 * CPT) + 4 * j + threadIdx.y;
    ok[j] = y < g.ny;
    idx[j] = x + g.nx * min(y, g.ny - 1) + plane * z;
  }
  float cx[CPT], cy[CPT], cz[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    cx[j] = ux[idx[j]];
    if (NDIM >= 2) cy[j] = uy[idx[j]];
    if (NDIM == 3) cz[j] = uz[idx[j]];
  }
  float v[CPT][8];
  bool over = false;  // an overflow, stored once below
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int y = min(blockIdx.y * (4 * CPT) + 4 * j + threadIdx.y, g.ny - 1);
    dx[j] = depart_o<R>(sgn * (cx[j] * g.lam[0]), over);
    const int xa = wrap1(x + dx[j].oa, g.nx), xb = wrap1(x + dx[j].ob, g.nx);
    if (NDIM == 1) {
      v[j][0] = a[xa];
      v[j][1] = a[xb];
      continue;
    }
    dy[j] = depart_o<R>(sgn * (cy[j] * g.lam[1]), over);
    const int ya = wrap1(y + dy[j].oa, g.ny) * g.nx, yb = wrap1(y + dy[j].ob, g.ny) * g.nx;
    int za = z * plane, zb = za;
    if (NDIM == 3) {
      dz[j] = depart_o<R>(sgn * (cz[j] * g.lam[2]), over);
      za = wrap1(z + dz[j].oa, g.nz) * plane;
      zb = wrap1(z + dz[j].ob, g.nz) * plane;
    }
    v[j][0] = a[za + ya + xa];
    v[j][1] = a[za + ya + xb];
    v[j][2] = a[za + yb + xa];
    v[j][3] = a[za + yb + xb];
    if (NDIM == 3) {
      v[j][4] = a[zb + ya + xa];
      v[j][5] = a[zb + ya + xb];
      v[j][6] = a[zb + yb + xa];
      v[j][7] = a[zb + yb + xb];
    }
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    float r;
    if (NDIM == 1) {
      r = lerp(v[j][0], v[j][1], dx[j].f);
    } else if (NDIM == 2) {
      r = lerp(lerp(v[j][0], v[j][1], dx[j].f), lerp(v[j][2], v[j][3], dx[j].f), dy[j].f);
    } else {
      const float v00 = lerp(v[j][0], v[j][1], dx[j].f);
      const float v10 = lerp(v[j][2], v[j][3], dx[j].f);
      const float v01 = lerp(v[j][4], v[j][5], dx[j].f);
      const float v11 = lerp(v[j][6], v[j][7], dx[j].f);
      r = lerp(lerp(v00, v10, dy[j].f), lerp(v01, v11, dy[j].f), dz[j].f);
    }
    if (MODE != 0) {
      const float bv = b[idx[j]];
      r = fmaf(0.5f, bv - r, MODE == 1 ? a[idx[j]] : bv);
    }
    if (ok[j]) out[idx[j]] = r;
  }
  if (over) *flag = 1;
}

// ---------------------------------------------------------------------------
// Unsplit FEC / BEC (eqs. intro:FEC, intro:BEC), all calls fused in one pass.
//
// A workgroup owns a TX x TY column of cells and marches along z over a chunk
// of planes.  Each stage keeps a ring of 2*RZ+1 planes in LDS:
//   stage 0  Phi                 halo K*R   (K = 2 for FEC, 3 for BEC)
//   stage 1  Phi1 = L_U Phi      halo (K-1)*R
//   stage 2  psi = Phi + (Phi - L_{-U} Phi1)/2       (BEC only)
//   output   FEC: Phi1 + (Phi - L_{-U} Phi1)/2 ;  BEC: L_U psi
// Stage k at plane p reads stage k-1 at planes p-RZ..p+RZ, so a stage lags
// its input by RZ planes and intermediates never leave LDS.
// ---------------------------------------------------------------------------
template <int NDIM, int SCHEME, int R, int TX, int TY>
struct EcShape {
  static constexpr int RY = NDIM >= 2 ? R : 0;
  static constexpr int RZ = NDIM == 3 ? R : 0;
  static constexpr int K = SCHEME == BEC ? 3 : 2;
  static constexpr int D = 2 * RZ + 1;
  static constexpr int HX(int k) { return (K - k) * R; }
  static constexpr int HY(int k) { return (K - k) * RY; }
  static constexpr int W(int k) { return TX + 2 * HX(k); }
  static constexpr int H(int k) { return TY + 2 * HY(k); }
  static constexpr int PLANE(int k) { return W(k) * H(k); }
  static constexpr int OFF(int k) { return k == 0 ? 0 : OFF(k - 1) + D * PLANE(k - 1); }
  static constexpr int FLOATS = OFF(K);
};

// Interpolate LDS stage array `src` (ring of D planes of W x H) at the
// departure cell of the point whose centre in src coordinates is (cx, cy) on
// local plane p.
template <int NDIM, int W, int PL, int D>
__device__ __forceinline__ float interp_lds(const float* src, int p, int cx, int cy,
                                            const Dep& dx, const Dep& dy, const Dep& dz) {
  const int xa = cx + dx.oa, xb = cx + dx.ob;
  if (NDIM == 1) {
    const float* r = src + (p % D) * PL + cy * W;
    return lerp(r[xa], r[xb], dx.f);
  }
  const int ya = (cy + dy.oa) * W, yb = (cy + dy.ob) * W;
  if (NDIM == 2) {
    const float* s = src + (p % D) * PL;
    return lerp(lerp(s[ya + xa], s[ya + xb], dx.f), lerp(s[yb + xa], s[yb + xb], dx.f), dy.f);
  }
  const float* sa = src + ((p + dz.oa) % D) * PL;
  const float* sb = src + ((p + dz.ob) % D) * PL;
  const float v00 = lerp(sa[ya + xa], sa[ya + xb], dx.f);
  const float v10 = lerp(sa[yb + xa], sa[yb + xb], dx.f);
  const float v01 = lerp(sb[ya + xa], sb[ya + xb], dx.f);
  const float v11 = lerp(sb[yb + xa], sb[yb + xb], dx.f);
  return lerp(lerp(v00, v10, dy.f), lerp(v01, v11, dy.f), dz.f);
}

template <int NDIM, int SCHEME, int R, int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_ec(const float* __restrict__ phi,
                                                 const float* __restrict__ ux,
                                                 const float* __restrict__ uy,
                                                 const float* __restrict__ uz,
                                                 float* __restrict__ out, Geo g, int zchunk,
                                                 int* flag) {
  using S = EcShape<NDIM, SCHEME, R, TX, TY>;
  constexpr int K = S::K, RZ = S::RZ, RY = S::RY, D = S::D;
  extern __shared__ float lds[];
  float* st0 = lds + S::OFF(0);
  float* st1 = lds + S::OFF(1);
  float* st2 = lds + S::OFF(K == 3 ? 2 : 1);  // psi (BEC only)

  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int zbeg = blockIdx.z * zchunk;
  const int zend = min(zbeg + zchunk, g.nz);
  const int first = zbeg - K * RZ;  // global plane of local plane 0
  const int iters = (zend - zbeg) + 2 * K * RZ;
  const int plane = g.nx * g.ny;

  // velocity and departures at global (x, y, z) for axis-wise offsets
  auto deps = [&](int gx, int gy, int gz, bool reverse, Dep& dx, Dep& dy, Dep& dz) {
    const size_t i = (size_t)gz * plane + (size_t)gy * g.nx + gx;
    float c = ux[i] * g.lam[0];
    dx = depart<R>(reverse ? -c : c, flag);
    if (NDIM >= 2) {
      c = uy[i] * g.lam[1];
      dy = depart<R>(reverse ? -c : c, flag);
    }
    if (NDIM == 3) {
      c = uz[i] * g.lam[2];
      dz = depart<R>(reverse ? -c : c, flag);
    }
  };

  for (int t = 0; t < iters; ++t) {
    // stage 0: load Phi plane (local t) with its halo
    {
      const int gz = wrapk(first + t, g.nz);
      float* dst = st0 + (t % D) * S::PLANE(0);
      constexpr int KL = (S::PLANE(0) + kThreads - 1) / kThreads;
      float v[KL];
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = threadIdx.x + k * kThreads;
        const int ly = e / S::W(0), lx = e - ly * S::W(0);
        const int gx = wrapk(x0 - S::HX(0) + lx, g.nx);
        const int gy = wrapk(y0 - S::HY(0) + ly, g.ny);
        v[k] = e < S::PLANE(0) ? phi[(size_t)gz * plane + (size_t)gy * g.nx + gx] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < KL; ++k) {
        const int e = threadIdx.x + k * kThreads;
        if (e < S::PLANE(0)) dst[e] = v[k];
      }
    }
    __syncthreads();
    // stage 1: Phi1 = L_U Phi at local plane t - RZ
    if (t >= 2 * RZ) {
      const int p = t - RZ;
      const int gz = wrapk(first + p, g.nz);
      float* dst = st1 + (p % D) * S::PLANE(1);
      for_strided<S::PLANE(1), kThreads>(threadIdx.x, [&](int e) {
        const int ly = e / S::W(1), lx = e - ly * S::W(1);
        const int gx = wrapk(x0 - S::HX(1) + lx, g.nx);
        const int gy = wrapk(y0 - S::HY(1) + ly, g.ny);
        Dep dx{}, dy{}, dz{};
        deps(gx, gy, gz, false, dx, dy, dz);
        dst[e] = interp_lds<NDIM, S::W(0), S::PLANE(0), D>(st0, p, lx + R, ly + RY, dx, dy, dz);
      });
    }
    __syncthreads();
    if (K == 3) {
      // stage 2 (BEC): psi = Phi + (Phi - L_{-U} Phi1)/2 at local plane t - 2RZ
      if (t >= 4 * RZ) {
        const int p = t - 2 * RZ;
        const int gz = wrapk(first + p, g.nz);
        float* dst = st2 + (p % D) * S::PLANE(2);
        const float* ph = st0 + (p % D) * S::PLANE(0);
        for_strided<S::PLANE(2), kThreads>(threadIdx.x, [&](int e) {
          const int ly = e / S::W(2), lx = e - ly * S::W(2);
          const int gx = wrapk(x0 - S::HX(2) + lx, g.nx);
          const int gy = wrapk(y0 - S::HY(2) + ly, g.ny);
          Dep dx{}, dy{}, dz{};
          deps(gx, gy, gz, true, dx, dy, dz);
          const float bar =
              interp_lds<NDIM, S::W(1), S::PLANE(1), D>(st1, p, lx + R, ly + RY, dx, dy, dz);
          const float v = ph[(ly + 2 * RY) * S::W(0) + lx + 2 * R];
          dst[e] = fmaf(0.5f, v - bar, v);
        });
      }
      __syncthreads();
    }
    // output at local plane t - K*RZ
    if (t >= 2 * K * RZ) {
      const int p = t - K * RZ;
      const int z = first + p;  // in [zbeg, zend)
      for_strided<TX * TY, kThreads>(threadIdx.x, [&](int e) {
        const int ly = e / TX, lx = e - ly * TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= g.nx || gy >= g.ny) return;
        float res;
        if (K == 2) {
          Dep dx{}, dy{}, dz{};
          deps(gx, gy, z, true, dx, dy, dz);
          const float bar =
              interp_lds<NDIM, S::W(1), S::PLANE(1), D>(st1, p, lx + R, ly + RY, dx, dy, dz);
          const float p1 = st1[(p % D) * S::PLANE(1) + (ly + RY) * S::W(1) + lx + R];
          const float v = st0[(p % D) * S::PLANE(0) + (ly + 2 * RY) * S::W(0) + lx + 2 * R];
          res = fmaf(0.5f, v - bar, p1);
        } else {
          Dep dx{}, dy{}, dz{};
          deps(gx, gy, z, false, dx, dy, dz);
          res = interp_lds<NDIM, S::W(2), S::PLANE(2), D>(st2, p, lx + R, ly + RY, dx, dy, dz);
        }
        out[(size_t)z * plane + (size_t)gy * g.nx + gx] = res;
      });
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Third-order sweep along one axis (eq. intro:CEC with eq. intro:CECcoef
// weights, large CFL per eq. intro:CECcoefSL; one axis at a time as in
// eqs. split:1-2).  Per node, with e = Phi - L_{-U} L_U Phi:
//   out = Phi1 + 1/2 [e_a + (1+f)/3 (e_b - e_a)],   Phi1 = L_U Phi,
// which for U < 1 is A FEC + B BEC with 3A = 2 - 1/U, B = 1 - A, written
// without the division.  A tile of TL nodes along the axis plus a halo of 3R
// (Phi), 2R (Phi1, Courant), R (e) is staged in LDS; the three calls never
// leave LDS.
// ---------------------------------------------------------------------------

// The last stage of a sweep, from Phi1 and e at the arrival node (ei) and at
// the anchor and far nodes of the departure interval (ea, eb).  COMB selects
// the scheme the sweep applies along its axis: the third order (lerp form of
// A FEC + B BEC), FEC (eq. intro:FEC: Phi1 + e/2 at the arrival node), BEC
// (eq. intro:BEC: L_U[Phi + e/2] = Phi1 + 1/2 [e_a + f (e_b - e_a)]) or the
// weights of eq. intro:CECcoefSL read literally, A FEC + B BEC with
// 3A = 2 - 1/f and B = 1 - A (f = |c| mod 1: second order beyond |c| = 1,
// not finite at f = 0), formed as B = 1 - A does: A (FEC - BEC) + BEC.
constexpr int kCombCec = 0, kCombFec = 1, kCombBec = 2, kCombCecLit = 3;
template <int COMB>
__device__ __forceinline__ float sweep_combine(float p1, float ei, float ea, float eb, float f) {
  if (COMB == kCombFec) return fmaf(0.5f, ei, p1);
  if (COMB == kCombCecLit) {
    const float a = (2.f - 1.f / f) / 3.f;
    const float fecv = fmaf(0.5f, ei, p1), becv = fmaf(0.5f, fmaf(f, eb - ea, ea), p1);
    return fmaf(a, fecv - becv, becv);
  }
  const float w = COMB == kCombBec ? f : fmaf(f, 1.f / 3.f, 1.f / 3.f);
  return fmaf(0.5f, fmaf(w, eb - ea, ea), p1);
}

// The Courant number at a midpoint of a node's backtrace (MID sweeps): the
// Courant numbers c of one column of a tile, cs apart in LDS, linearly
// interpolated at local position pos (within the column: callers keep pos
// at least one node inside it).
__device__ __forceinline__ float mid_courant(const float* c, int cs, float pos, int nmax) {
  float i0f = floorf(pos);
  const float fr = pos - i0f;
  const int i0 = min(max(int(i0f), 0), nmax - 2);
  return (1.f - fr) * c[i0 * cs] + fr * c[(i0 + 1) * cs];
}

// Strided axis (y or z): tile = 64 consecutive x (coalesced) x TL along the axis.
// MID: a midpoint backtrace (beyond the paper): the calls of L_U depart
// from x - c(x - c/2) and the call of L_{-U} from x + c(x + c/2), the
// Courant numbers interpolated along the axis from the tile's own, which
// then reach 3R nodes out like phi.
template <int R, int COMB = kCombCec, bool MID = false>
__global__ __launch_bounds__(kThreads) void k_sweep_s(const float* __restrict__ phi,
                                                      const float* __restrict__ ud,
                                                      float* __restrict__ out, int nx, int L,
                                                      int64_t S, int64_t So, float lam, int* flag) {
  constexpr int TL = 32, TW = 64;
  constexpr int NP = TL + 6 * R, NC = TL + 4 * R, NE = TL + 2 * R;
  constexpr int NL = MID ? NP : NC, CO = MID ? 3 * R : 2 * R;  // Courant rows loaded, their start
  __shared__ float P[NP * TW], C[NL * TW], P1[NC * TW], E[NE * TW];
  __shared__ float CM[MID ? 2 * NC * TW : 1];  // midpoint Courant numbers: forward, then reverse
  const int tx = threadIdx.x & (TW - 1), ty = threadIdx.x / TW;
  const int x = blockIdx.x * TW + tx;
  const int l0 = blockIdx.y * TL;
  const bool xin = x < nx;
  const size_t base = (size_t)blockIdx.z * So + (xin ? x : 0);
  // issue every load of the tile before the first LDS store
  constexpr int RS = kThreads / TW;  // rows per pass
  constexpr int KPr = (NP + RS - 1) / RS, KCr = (NL + RS - 1) / RS;
  float vp[KPr], vc[KCr];
#pragma unroll
  for (int k = 0; k < KPr; ++k) {
    const int r = ty + k * RS;
    const int l = wrapk(l0 - 3 * R + r, L);
    vp[k] = (xin && r < NP) ? phi[base + (size_t)l * S] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < KCr; ++k) {
    const int r = ty + k * RS;
    const int l = wrapk(l0 - CO + r, L);
    vc[k] = (xin && r < NL) ? ud[base + (size_t)l * S] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < KPr; ++k)
    if (ty + k * RS < NP) P[(ty + k * RS) * TW + tx] = vp[k];
#pragma unroll
  for (int k = 0; k < KCr; ++k)
    if (ty + k * RS < NL) C[(ty + k * RS) * TW + tx] = vc[k] * lam;
  __syncthreads();
  // forward and reverse Courant numbers of the tile's nodes a0 - 2R + r
  const float* CF = MID ? CM : C;
  const float* CB = MID ? CM + NC * TW : C;
  if (MID) {
    for_strided<NC, kThreads / TW>(ty, [&](int r) {
      const float c = C[(r + R) * TW + tx];
      CM[r * TW + tx] = mid_courant(C + tx, TW, float(r + R) - 0.5f * c, NL);
      CM[(NC + r) * TW + tx] = mid_courant(C + tx, TW, float(r + R) + 0.5f * c, NL);
    });
    __syncthreads();
  }
  for_strided<NC, kThreads / TW>(ty, [&](int r) {
    const Dep d = depart<R>(CF[r * TW + tx], flag);
    P1[r * TW + tx] = lerp(P[(r + R + d.oa) * TW + tx], P[(r + R + d.ob) * TW + tx], d.f);
  });
  __syncthreads();
  for_strided<NE, kThreads / TW>(ty, [&](int r) {
    const Dep d = depart<R>(-CB[(r + R) * TW + tx], flag);
    const float bar = lerp(P1[(r + R + d.oa) * TW + tx], P1[(r + R + d.ob) * TW + tx], d.f);
    E[r * TW + tx] = P[(r + 2 * R) * TW + tx] - bar;
  });
  __syncthreads();
  if (!xin) return;
  for_strided<TL, kThreads / TW>(ty, [&](int r) {
    const int l = l0 + r;
    if (l >= L) return;
    const Dep d = depart<R>(CF[(r + 2 * R) * TW + tx], flag);
    const float ea = E[(r + R + d.oa) * TW + tx], eb = E[(r + R + d.ob) * TW + tx];
    out[base + (size_t)l * S] =
        sweep_combine<COMB>(P1[(r + 2 * R) * TW + tx], E[(r + R) * TW + tx], ea, eb, d.f);
  });
}

// Contiguous axis (x): tile = TL consecutive x in each of ROWS rows.  MID
// as in k_sweep_s.
template <int R, int COMB = kCombCec, bool MID = false>
__global__ __launch_bounds__(kThreads) void k_sweep_x(const float* __restrict__ phi,
                                                      const float* __restrict__ ud,
                                                      float* __restrict__ out, int nx, int ny,
                                                      float lam, int* flag) {
  constexpr int TL = 256, ROWS = 4;
  constexpr int NP = TL + 6 * R, NC = TL + 4 * R, NE = TL + 2 * R;
  constexpr int NL = MID ? NP : NC, CO = MID ? 3 * R : 2 * R;  // Courant entries loaded, their start
  __shared__ float P[ROWS * NP], C[ROWS * NL], P1[ROWS * NC], E[ROWS * NE];
  __shared__ float CM[MID ? 2 * ROWS * NC : 1];  // midpoint Courant numbers: forward, then reverse
  const int l0 = blockIdx.x * TL;
  const int y0 = blockIdx.y * ROWS;
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  // issue every load of the tile before the first LDS store
  constexpr int KPe = (ROWS * NP + kThreads - 1) / kThreads;
  constexpr int KCe = (ROWS * NL + kThreads - 1) / kThreads;
  float vp[KPe], vc[KCe];
#pragma unroll
  for (int k = 0; k < KPe; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int rr = e / NP, col = e - rr * NP;
    const int y = y0 + rr;
    vp[k] = (e < ROWS * NP && y < ny) ? phi[zoff + (size_t)y * nx + wrapk(l0 - 3 * R + col, nx)] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < KCe; ++k) {
    const int e = threadIdx.x + k * kThreads;
    const int rr = e / NL, col = e - rr * NL;
    const int y = y0 + rr;
    vc[k] = (e < ROWS * NL && y < ny) ? ud[zoff + (size_t)y * nx + wrapk(l0 - CO + col, nx)] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < KPe; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < ROWS * NP) P[e] = vp[k];
  }
#pragma unroll
  for (int k = 0; k < KCe; ++k) {
    const int e = threadIdx.x + k * kThreads;
    if (e < ROWS * NL) C[e] = vc[k] * lam;
  }
  __syncthreads();
  // forward and reverse Courant numbers of node l0 - 2R + col of row rr at
  // rr * NC + col
  const float* CF = MID ? CM : C;
  const float* CB = MID ? CM + ROWS * NC : C;
  if (MID) {
    for_strided<ROWS * NC, kThreads>(threadIdx.x, [&](int e) {
      const int rr = e / NC, col = e - rr * NC;
      const float* row = C + rr * NL;
      const float c = row[col + R];
      CM[e] = mid_courant(row, 1, float(col + R) - 0.5f * c, NL);
      CM[ROWS * NC + e] = mid_courant(row, 1, float(col + R) + 0.5f * c, NL);
    });
    __syncthreads();
  }
  for_strided<ROWS * NC, kThreads>(threadIdx.x, [&](int e) {
    const int rr = e / NC, col = e - rr * NC;
    const Dep d = depart<R>(CF[e], flag);
    const float* p = P + rr * NP + col + R;
    P1[e] = lerp(p[d.oa], p[d.ob], d.f);
  });
  __syncthreads();
  for_strided<ROWS * NE, kThreads>(threadIdx.x, [&](int e) {
    const int rr = e / NE, col = e - rr * NE;
    const Dep d = depart<R>(-CB[rr * NC + col + R], flag);
    const float* p1 = P1 + rr * NC + col + R;
    E[e] = P[rr * NP + col + 2 * R] - lerp(p1[d.oa], p1[d.ob], d.f);
  });
  __syncthreads();
  for_strided<ROWS * TL, kThreads>(threadIdx.x, [&](int e) {
    const int rr = e / TL, col = e - rr * TL;
    const int y = y0 + rr, x = l0 + col;
    if (y >= ny || x >= nx) return;
    const Dep d = depart<R>(CF[rr * NC + col + 2 * R], flag);
    const float* ee = E + rr * NE + col + R;
    out[zoff + (size_t)y * nx + x] =
        sweep_combine<COMB>(P1[rr * NC + col + 2 * R], ee[0], ee[d.oa], ee[d.ob], d.f);
  });
}

// ---------------------------------------------------------------------------
// Marching sweep along a strided axis (y or z), any reach R.  A thread owns
// V = 1 or 2 neighbouring columns (x from the lane, the other strided
// coordinate from the workgroup; V = 2 with even nx: one 8-byte access per
// row) and walks along the sweep axis over positions m = l0 - 3R ..
// l1 - 1 + 3R, loading phi and the velocity once per node.  At step m:
//   Phi1 of node m - R  (needs phi of m - 2R .. m),
//   e    of node m - 2R (needs Phi1 of m - 3R .. m - R),
//   out  of node m - 3R (needs e of m - 4R .. m - 2R).
// Rings of K = 3R + 1 registers hold phi, Phi1, e and the Courant numbers,
// node n at index (n - l0 + 3R) mod K; the walk is unrolled by K so that
// every ring index is a compile-time constant.  Loads run K steps ahead
// into a second register set.  Addresses are a per-thread byte offset plus
// a row offset that is the same for the whole wave (a scalar register), so
// a load or store needs no vector instruction.  No LDS and no barriers.
// The arithmetic per node is that of k_sweep_s.  Fields of at most 2^30
// cells (32-bit byte offsets).
// ---------------------------------------------------------------------------
// Access at a per-thread byte offset voff from the row or plane that starts
// soff bytes into the field (soff the same for the whole wave): a buffer
// descriptor rebased on that row or plane (two scalar adds), with the
// largest size a descriptor holds, so only voff is range-checked.  A
// descriptor on the field's start cannot cover a field of 2^30 cells (its
// size tops out one byte short of 2^32 and would clip the last element).
// voff + 4 stays below 2^32 when ny >= 2 or the field holds fewer than 2^30
// cells (the launchers check that).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc based_rsrc(const float* field, unsigned soff) {
  // readfirstlane returns a signed int: widen the byte offset as unsigned
  const size_t off = unsigned(__builtin_amdgcn_readfirstlane(int(soff)));
  const char* b = reinterpret_cast<const char*>(field) + off;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), short(0), int(0xFFFFFFFFu), 0x00020000);
}
__device__ __forceinline__ float ld_row(const float* field, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_raw_buffer_load_b32(based_rsrc(field, soff), voff, 0, 0));
}
__device__ __forceinline__ void st_row(float* field, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), based_rsrc(field, soff), voff,
                                        0, 0);
}
// Two consecutive nodes at an 8-byte aligned voff.
// The 64-bit builtins' type is cast whole to a float pair: bit-casting its
// integer elements one by one compiled to a 32-bit load whose value served
// both nodes.
typedef unsigned b64v __attribute__((ext_vector_type(2)));  // the 64-bit buffer builtins' type
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void ld2_row(const float* field, unsigned voff, unsigned soff, float& a,
                                        float& b) {
  const f2v v = __builtin_bit_cast(
      f2v, __builtin_amdgcn_raw_buffer_load_b64(based_rsrc(field, soff), voff, 0, 0));
  a = v.x;
  b = v.y;
}
__device__ __forceinline__ void st2_row(float* field, unsigned voff, unsigned soff, float a, float b) {
  const f2v v = {a, b};
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64v, v), based_rsrc(field, soff), voff, 0,
                                        0);
}

// V = 1 or 2 consecutive nodes
template <int V>
__device__ __forceinline__ void ld_rowv(const float* field, unsigned voff, unsigned soff,
                                        float (&o)[V]) {
  if constexpr (V == 1)
    o[0] = ld_row(field, voff, soff);
  else
    ld2_row(field, voff, soff, o[0], o[1]);
}
template <int V>
__device__ __forceinline__ void st_rowv(float* field, unsigned voff, unsigned soff,
                                        const float (&o)[V]) {
  if constexpr (V == 1)
    st_row(field, voff, soff, o[0]);
  else
    st2_row(field, voff, soff, o[0], o[1]);
}

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int pmod(int a, int k) { return ((a % k) + k) % k; }

// Departure of a node as anchor direction and distance (the decomposition
// of depart<R>, same clamp): anchor = node - n if pos, node + n otherwise;
// far = one further.  An overflow is recorded in *over*, which the kernel
// stores to the flag once at its end: a store under a condition at every
// departure costs a branch per call.
struct DepN {
  float f;
  float n;  // a whole number, compared as a float (no conversion)
  bool pos;
};
template <int R>
__device__ __forceinline__ DepN depart_n(float c, bool& over) {
  const float mag = fabsf(c);
  const float nf = floorf(mag);
  const float f = mag - nf;
  over |= nf > float(R - 1);  // false for NaN, which propagates
  return DepN{f, fminf(nf, float(R - 1)), c >= 0.f};
}
// The fraction and clamped distance of a Courant number, shared by the
// forward and the reverse departure (|c| is the same); the ring marches
// keep them per ring slot, computed once per row.
template <int R>
__device__ __forceinline__ void depart_fn(float c, float& f, float& n, bool& over) {
  const float mag = fabsf(c);
  const float nf = floorf(mag);
  f = mag - nf;
  over |= nf > float(R - 1);
  n = fminf(nf, float(R - 1));
}
// forward (depart_n(c)) and reverse (depart_n(-c)) from them: -c >= 0 is
// c <= 0 (both false for NaN; -0.0 >= 0 holds)
__device__ __forceinline__ DepN dep_fwd(float c, float f, float n) { return DepN{f, n, c >= 0.f}; }
__device__ __forceinline__ DepN dep_rev(float c, float f, float n) { return DepN{f, n, c <= 0.f}; }

// A value passed through an empty asm statement: the compiler cannot move
// an operation on it to where v was produced.  The ring marches pass their
// prefetched values through it where they are used (see k_sweep_m).
__device__ __forceinline__ float opaque(float v) {
  asm("" : "+v"(v));
  return v;
}

// Anchor and far values of a call at ring index BASE: the anchor at
// distance n from the node, the far value at n + 1, both on the side the
// departure lies (pos: lower indices).  The side is chosen first for each
// distance (R selects), then the distance (2(R - 1) selects): 3R - 2 in
// all, against 4R - 2 choosing the distance first.
template <int R, int K, int BASE>
__device__ __forceinline__ void ring_pair(const float (&ring)[K], const DepN& d, float& a, float& b) {
  float v[R + 1];  // v[k]: the candidate at distance k on the departure's side
  v[0] = ring[pmod(BASE, K)];
#pragma unroll
  for (int k = 1; k <= R; ++k) v[k] = d.pos ? ring[pmod(BASE - k, K)] : ring[pmod(BASE + k, K)];
  a = v[0];
  b = v[1];
#pragma unroll
  for (int k = 1; k < R; ++k) {
    const bool hit = d.n == float(k);
    a = hit ? v[k] : a;
    b = hit ? v[k + 1] : b;
  }
}

template <int R, int V, int COMB = kCombCec>
__global__ __launch_bounds__(kThreads) void k_sweep_m(const float* __restrict__ phi,
                                                      const float* __restrict__ ud,
                                                      float* __restrict__ out, int nx, int L,
                                                      unsigned S4, unsigned So4, int nother,
                                                      int chunk, float lam, int* flag) {
  constexpr int K = 3 * R + 1;
  const int x = blockIdx.x * (64 * V) + V * (threadIdx.x & 63);  // the lane's first column
  const int other = blockIdx.y * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (x >= nx || other >= nother) return;
  const int l0 = blockIdx.z * chunk;
  const int l1 = min(l0 + chunk, L);
  const unsigned voff = 4u * unsigned(x) + unsigned(other) * So4;
  const float *rp = phi, *ru = ud;
  float* ro = out;
  auto wrapped = [&](int m) {
    m %= L;
    return m < 0 ? m + L : m;
  };
  const int m0 = l0 - 3 * R, m1 = l1 + 3 * R;  // steps m0 .. m1 - 1
  // loads run PD steps ahead: K, or K/2 for two columns at reach 3 (20
  // registers fewer, as in k_sweep_xyp)
  constexpr int PD = (R == 3 && V == 2) ? K / 2 : K;
  static_assert(K % PD == 0, "prefetch slots are ring indices mod PD");
  float pr[V][K], p1[V][K], er[V][K], cr[V][K];  // rings, per column
  float fr[V][K], nr[V][K];  // departure fraction and distance of each ring slot
  float np[V][PD], nc[V][PD];  // loads of the next PD steps
  int lrow = wrapped(m0);    // wrapped axis position of the next load
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int v = 0; v < V; ++v) pr[v][i] = p1[v][i] = er[v][i] = cr[v][i] = fr[v][i] = nr[v][i] = 0.f;
#pragma unroll
  for (int i = 0; i < PD; ++i) {
    const unsigned ro_i = unsigned(lrow) * S4;
    float a[V], c[V];
    ld_rowv<V>(rp, voff, ro_i, a);
    ld_rowv<V>(ru, voff, ro_i, c);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      np[v][i] = a[v];
      nc[v][i] = c[v];
    }
    lrow = lrow + 1 == L ? 0 : lrow + 1;
    // issued in step order: the loop's first step then waits for the
    // oldest loads only
    __builtin_amdgcn_sched_barrier(0);
  }
  int srow = wrapped(m0 - 3 * R);  // wrapped axis position of node m - 3R
  bool over = false;
  for (int mb = m0; mb < m1; mb += K) {
    static_for<K>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int m = mb + i;
      constexpr int q = i % PD;  // prefetch slot of this step
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // the loaded values pass through opaque() where they are used: the
        // compiler would otherwise move these products into the previous
        // iteration, right after the loads, and wait for them there
        pr[v][i] = opaque(np[v][q]);
        cr[v][i] = opaque(nc[v][q]) * lam;
        depart_fn<R>(cr[v][i], fr[v][i], nr[v][i], over);
      }
      {  // unconditional, and every iteration runs all K steps (past m1 the
         // loads read wrapped rows whose results go unused): a load under a
         // condition makes the wave wait for the loads in flight
        const unsigned rn = unsigned(lrow) * S4;
        float a[V], c[V];
        ld_rowv<V>(rp, voff, rn, a);
        ld_rowv<V>(ru, voff, rn, c);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          np[v][q] = a[v];
          nc[v][q] = c[v];
        }
      }
      lrow = lrow + 1 == L ? 0 : lrow + 1;
      constexpr int j1 = pmod(i - R, K), j2 = pmod(i - 2 * R, K), j3 = pmod(i - 3 * R, K);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        {  // Phi1 of node m - R
          const DepN d = dep_fwd(cr[v][j1], fr[v][j1], nr[v][j1]);
          float a, b;
          ring_pair<R, K, j1>(pr[v], d, a, b);
          p1[v][j1] = lerp(a, b, d.f);
        }
        {  // e of node m - 2R
          const DepN d = dep_rev(cr[v][j2], fr[v][j2], nr[v][j2]);
          float a, b;
          ring_pair<R, K, j2>(p1[v], d, a, b);
          er[v][j2] = pr[v][j2] - lerp(a, b, d.f);
        }
      }
      // out of node m - 3R
      if (m - 3 * R >= l0 && m - 3 * R < l1) {
        float o[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const DepN d = dep_fwd(cr[v][j3], fr[v][j3], nr[v][j3]);
          float ea, eb;
          ring_pair<R, K, j3>(er[v], d, ea, eb);
          o[v] = sweep_combine<COMB>(p1[v][j3], er[v][j3], ea, eb, d.f);
        }
        st_rowv<V>(ro, voff, unsigned(srow) * S4, o);
      }
      srow = srow + 1 == L ? 0 : srow + 1;
    });
  }
  if (over) *flag = 1;
}

// ---------------------------------------------------------------------------
// Window sweep along x, any reach R.  A window is 64 consecutive x of one
// row, x0 - 3R .. x0 + 60 - 3R (wrapped), one node per lane; a wave loads 4
// consecutive windows of its row together.  A window
// produces the 64 - 6R outputs x0 .. x0 + 63 - 6R; the anchor and far
// values of each call are read from the lanes at the departure offsets
// (xsweep_lanes: DPP shifts at reach 1 and 2, __shfl beyond): Phi1 is valid
// on lanes R .. 63 - R, e on 2R .. 63 - 2R, the output on 3R .. 63 - 3R.
// No LDS memory, no barriers.  The arithmetic per node is that of k_sweep_x
// (COMB: the scheme applied along the axis, as there).
// ---------------------------------------------------------------------------
// Value of the lane below (lane - 1) and above (lane + 1): DPP wave shifts,
// one vector move each; lanes 0 and 63 receive 0.
__device__ __forceinline__ float lane_below(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, i, 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_above(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, i, 0x130, 0xf, 0xf, true));
}

// Anchor and far values of a call from the values of the lanes k = 0 .. R
// below (lo[k]) and above (hi[k]): the selection of ring_pair.
template <int R>
__device__ __forceinline__ void view_pair(const float (&lo)[R + 1], const float (&hi)[R + 1],
                                          const DepN& d, float& a, float& b) {
  float v[R + 1];
  v[0] = lo[0];
#pragma unroll
  for (int k = 1; k <= R; ++k) v[k] = d.pos ? lo[k] : hi[k];
  a = v[0];
  b = v[1];
#pragma unroll
  for (int k = 1; k < R; ++k) {
    const bool hit = d.n == float(k);
    a = hit ? v[k] : a;
    b = hit ? v[k + 1] : b;
  }
}
template <int R>
__device__ __forceinline__ void lane_views(float v, float (&lo)[R + 1], float (&hi)[R + 1]) {
  lo[0] = hi[0] = v;
#pragma unroll
  for (int k = 1; k <= R; ++k) {
    lo[k] = lane_below(lo[k - 1]);
    hi[k] = lane_above(hi[k - 1]);
  }
}

// Third-order sweep along x of one value per lane (lanes are consecutive
// x): the anchor and far values of each call come from the lanes at the
// departure offsets, by DPP shifts at reach 1 and 2 (2R vector moves per
// value, no LDS) and by __shfl (a cross-lane read through LDS hardware)
// beyond.  Exact on lanes 3R .. 63 - 3R; an overflow is recorded in over.
template <int R, int COMB = kCombCec>
__device__ __forceinline__ float xsweep_lanes(float p, float c, int lane, bool& over) {
  const DepN d = depart_n<R>(c, over), dr = depart_n<R>(-c, over);
  float p1, e, ea, eb;
  if constexpr (R <= 2) {
    float lo[R + 1], hi[R + 1], a, b;
    lane_views<R>(p, lo, hi);
    view_pair<R>(lo, hi, d, a, b);
    p1 = lerp(a, b, d.f);
    lane_views<R>(p1, lo, hi);
    view_pair<R>(lo, hi, dr, a, b);
    e = p - lerp(a, b, dr.f);
    lane_views<R>(e, lo, hi);
    view_pair<R>(lo, hi, d, ea, eb);
  } else {
    const int n = int(d.n), nr = int(dr.n);
    const int oa = d.pos ? -n : n, ob = d.pos ? -(n + 1) : n + 1;
    const int ra = dr.pos ? -nr : nr, rb = dr.pos ? -(nr + 1) : nr + 1;
    p1 = lerp(__shfl(p, lane + oa), __shfl(p, lane + ob), d.f);
    e = p - lerp(__shfl(p1, lane + ra), __shfl(p1, lane + rb), dr.f);
    ea = __shfl(e, lane + oa);
    eb = __shfl(e, lane + ob);
  }
  return sweep_combine<COMB>(p1, e, ea, eb, d.f);
}

template <int R, int COMB = kCombCec>
__global__ __launch_bounds__(kThreads) void k_sweep_xw(const float* __restrict__ phi,
                                                       const float* __restrict__ ud,
                                                       float* __restrict__ out, int nx, int nrows,
                                                       int nwin, float lam, int* flag) {
  constexpr int USE = 64 - 6 * R;  // outputs per window
  constexpr int WPW = 4;           // windows per wave, loaded together
  const int lane = threadIdx.x & 63;
  // the wave's index, in a scalar register (row arithmetic stays scalar)
  const int wid = blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ngrp = (nwin + WPW - 1) / WPW;
  bool over = false;
  const int row = wid / ngrp;
  if (row >= nrows) return;
  const int w0 = (wid - row * ngrp) * WPW;
  const unsigned rowoff = 4u * unsigned(row) * unsigned(nx);  // the same for the whole wave
  unsigned off[WPW];
  float p[WPW], c[WPW];
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    const int x = wrapk((w0 + k) * USE - 3 * R + lane, nx);
    off[k] = 4u * unsigned(x);
    p[k] = c[k] = 0.f;
    if (w0 + k < nwin) {  // the same for the whole wave
      p[k] = ld_row(phi, off[k], rowoff);
      c[k] = ld_row(ud, off[k], rowoff);
    }
  }
#pragma unroll
  for (int k = 0; k < WPW; ++k) {
    if (w0 + k >= nwin) break;
    const float o = xsweep_lanes<R, COMB>(p[k], c[k] * lam, lane, over);
    const int xo = (w0 + k) * USE + lane - 3 * R;  // output node of this lane
    if (lane >= 3 * R && lane < 64 - 3 * R && xo < nx) st_row(out, off[k], rowoff, o);
  }
  if (over) *flag = 1;
}

// ---------------------------------------------------------------------------
// Fused x and y sweeps, reach 1 or 2 (odd nx; even nx takes k_sweep_xyp):
// the first two sweeps of an x,y,z step (XFIRST: x then y) or the last two
// of a z,y,x step (y then x), COMB the scheme along each axis.  A wave
// takes one 64-lane x window of one z plane, x0 - 3R .. x0 + 60 - 3R
// (wrapped, one node per lane; lanes 3R .. 63 - 3R are its 64 - 6R
// outputs), and marches along y through a chunk of rows with the y sweep's
// stencil in rings of K = 3R + 1 registers, as k_sweep_m does.  XFIRST:
// every loaded row is swept along x across the lanes (xsweep_lanes) before
// it enters the rings.  Otherwise every output row of the y sweep is swept
// along x.  The y sweep works lane by lane, so the lanes whose x sweep is
// exact give exact results.  The four waves of a workgroup take four
// neighbouring windows of one row, which share the lines their lane halos
// straddle.  Loads and stores address a row through a descriptor rebased
// on it, with the lane's x offset.  The same FP32 operations per node as
// k_sweep_xw followed by k_sweep_m (or the reverse).  Phi and the two
// velocity planes are read once and Phi written once: 16 B per node
// instead of 24 for the two sweeps.
// ---------------------------------------------------------------------------
template <int R, bool XFIRST, int COMB = kCombCec>
__global__ __launch_bounds__(kThreads) void k_sweep_xym(const float* __restrict__ phi,
                                                        const float* __restrict__ ux,
                                                        const float* __restrict__ uy,
                                                        float* __restrict__ out, int nx, int ny,
                                                        int nz, int nwin, int chunk, float lamx,
                                                        float lamy, int* flag) {
  constexpr int K = 3 * R + 1;
  constexpr int USE = 64 - 6 * R;  // outputs per window
  const int lane = threadIdx.x & 63;
  // the wave's index, in a scalar register (row arithmetic stays scalar)
  const int wid = blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int win = wid % nwin, z = (wid / nwin) % nz, ch = wid / (nwin * nz);
  const int l0 = ch * chunk;
  if (l0 >= ny) return;  // the whole wave
  const int l1 = min(l0 + chunk, ny);
  const unsigned vx = 4u * unsigned(wrapk(win * USE - 3 * R + lane, nx));
  const unsigned rowb = 4u * unsigned(nx);
  const unsigned zoff = unsigned(z) * unsigned(ny) * rowb;  // the plane's byte offset
  const bool lane_out = lane >= 3 * R && lane < 64 - 3 * R && win * USE + lane - 3 * R < nx;
  auto wrapped = [&](int m) {
    m %= ny;
    return m < 0 ? m + ny : m;
  };
  const int m0 = l0 - 3 * R, m1 = l1 + 3 * R;  // steps m0 .. m1 - 1
  float pr[K], p1[K], er[K], cr[K];  // rings
  float fr[K], nr[K];                // departure fraction and distance of each ring slot
  float np[K], nc[K], nx_[K];        // loads of the next K steps (nx_: x velocity)
  int lrow = wrapped(m0);            // row of the next phi / y-velocity load
  int xrow = XFIRST ? lrow : wrapped(m0 - 3 * R);  // row of the next x-velocity load
#pragma unroll
  for (int i = 0; i < K; ++i) {
    pr[i] = p1[i] = er[i] = cr[i] = fr[i] = nr[i] = 0.f;
    const unsigned ro = zoff + unsigned(lrow) * rowb;
    np[i] = ld_row(phi, vx, ro);
    nc[i] = ld_row(uy, vx, ro);
    nx_[i] = ld_row(ux, vx, zoff + unsigned(xrow) * rowb);
    lrow = lrow + 1 == ny ? 0 : lrow + 1;
    xrow = xrow + 1 == ny ? 0 : xrow + 1;
    __builtin_amdgcn_sched_barrier(0);  // in step order, as in k_sweep_m
  }
  int srow = wrapped(m0 - 3 * R);  // row of node m - 3R
  bool over = false;
  for (int mb = m0; mb < m1; mb += K) {
    static_for<K>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int m = mb + i;
      // the loaded values pass through opaque() where they are used: the
      // compiler would otherwise move these products into the previous
      // iteration, right after the loads, and wait for them there
      const float cx = opaque(nx_[i]) * lamx;  // x Courant number of row m (XFIRST) or of row m - 3R
      pr[i] = XFIRST ? xsweep_lanes<R, COMB>(opaque(np[i]), cx, lane, over) : opaque(np[i]);
      cr[i] = opaque(nc[i]) * lamy;
      depart_fn<R>(cr[i], fr[i], nr[i], over);
      {  // unconditional, all K steps, as in k_sweep_m
        const unsigned rn = zoff + unsigned(lrow) * rowb;
        np[i] = ld_row(phi, vx, rn);
        nc[i] = ld_row(uy, vx, rn);
        nx_[i] = ld_row(ux, vx, zoff + unsigned(xrow) * rowb);
      }
      lrow = lrow + 1 == ny ? 0 : lrow + 1;
      xrow = xrow + 1 == ny ? 0 : xrow + 1;
      // Phi1 of node m - R
      constexpr int j1 = pmod(i - R, K);
      {
        const DepN d = dep_fwd(cr[j1], fr[j1], nr[j1]);
        float a, b;
        ring_pair<R, K, j1>(pr, d, a, b);
        p1[j1] = lerp(a, b, d.f);
      }
      // e of node m - 2R
      constexpr int j2 = pmod(i - 2 * R, K);
      {
        const DepN d = dep_rev(cr[j2], fr[j2], nr[j2]);
        float a, b;
        ring_pair<R, K, j2>(p1, d, a, b);
        er[j2] = pr[j2] - lerp(a, b, d.f);
      }
      // out of node m - 3R
      constexpr int j3 = pmod(i - 3 * R, K);
      if (m - 3 * R >= l0 && m - 3 * R < l1) {
        const DepN d = dep_fwd(cr[j3], fr[j3], nr[j3]);
        float ea, eb;
        ring_pair<R, K, j3>(er, d, ea, eb);
        float o = sweep_combine<COMB>(p1[j3], er[j3], ea, eb, d.f);
        if (!XFIRST) o = xsweep_lanes<R, COMB>(o, cx, lane, over);
        if (lane_out) st_row(out, vx, zoff + unsigned(srow) * rowb, o);
      }
      srow = srow + 1 == ny ? 0 : srow + 1;
    });
  }
  if (over) *flag = 1;
}

// ---------------------------------------------------------------------------
// The fused x and y sweeps of k_sweep_xym with two nodes per lane, for even
// nx: a wave's window is 128 consecutive x of one z plane (lane l: nodes 2l
// and 2l+1, one 8-byte access), HL = 3R rounded up to even nodes of halo
// on each side, and up to 128 - 2 HL outputs.  The windows of a row are
// balanced (usew outputs each, even, the last one shorter); lanes past the
// nodes a window needs repeat its last pair, so every load is unconditional
// and reads no line twice.  Pairs start on even x and never straddle the
// periodic end.  Per node the same FP32 operations as k_sweep_xym, which
// this kernel matches bit for bit; the halo costs 2 HL / usew of the loads
// instead of 6R / (64 - 6R).
// ---------------------------------------------------------------------------
// Values at distance k = 0 .. R below (l*) and above (h*) nodes a = 2l and
// b = 2l + 1 of a row held as pairs: node 2l - 1 is lane l-1's b, 2l + 2
// lane l+1's a, and so on (DPP wave shifts; R <= 3).
template <int R>
__device__ __forceinline__ void pair_views(float a, float b, float (&la)[R + 1], float (&ha)[R + 1],
                                           float (&lb)[R + 1], float (&hb)[R + 1]) {
  static_assert(R >= 1 && R <= 3, "pair views reach three nodes");
  const float ba = lane_below(a), bb = lane_below(b), aa = lane_above(a), ab = lane_above(b);
  la[0] = ha[0] = a;
  lb[0] = hb[0] = b;
  la[1] = bb;
  ha[1] = b;
  lb[1] = a;
  hb[1] = aa;
  if constexpr (R >= 2) {
    la[2] = ba;
    ha[2] = aa;
    lb[2] = bb;
    hb[2] = ab;
  }
  if constexpr (R >= 3) {
    la[3] = lane_below(bb);
    ha[3] = ab;
    lb[3] = ba;
    hb[3] = lane_above(aa);
  }
}

// xsweep_lanes for a row held as pairs: the same operations per node.
template <int R, int COMB = kCombCec>
__device__ __forceinline__ void xsweep_pair(float& a, float& b, float ca, float cb, bool& over) {
  const DepN da = depart_n<R>(ca, over), ra = depart_n<R>(-ca, over);
  const DepN db = depart_n<R>(cb, over), rb = depart_n<R>(-cb, over);
  float la[R + 1], ha[R + 1], lb[R + 1], hb[R + 1], u, v;
  pair_views<R>(a, b, la, ha, lb, hb);
  view_pair<R>(la, ha, da, u, v);
  const float p1a = lerp(u, v, da.f);
  view_pair<R>(lb, hb, db, u, v);
  const float p1b = lerp(u, v, db.f);
  pair_views<R>(p1a, p1b, la, ha, lb, hb);
  view_pair<R>(la, ha, ra, u, v);
  const float ea = a - lerp(u, v, ra.f);
  view_pair<R>(lb, hb, rb, u, v);
  const float eb = b - lerp(u, v, rb.f);
  pair_views<R>(ea, eb, la, ha, lb, hb);
  view_pair<R>(la, ha, da, u, v);
  a = sweep_combine<COMB>(p1a, ea, u, v, da.f);
  view_pair<R>(lb, hb, db, u, v);
  b = sweep_combine<COMB>(p1b, eb, u, v, db.f);
}

template <int R>
constexpr int pair_halo() { return (3 * R + 1) / 2 * 2; }  // 3R rounded up to even

template <int R, bool XFIRST, int COMB = kCombCec>
__global__ __launch_bounds__(kThreads) void k_sweep_xyp(const float* __restrict__ phi,
                                                        const float* __restrict__ ux,
                                                        const float* __restrict__ uy,
                                                        float* __restrict__ out, int nx, int ny,
                                                        int nz, int nwin, int usew, int chunk,
                                                        float lamx, float lamy, int* flag) {
  constexpr int K = 3 * R + 1;
  constexpr int HL = pair_halo<R>();
  const int lane = threadIdx.x & 63;
  const int wid = blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int win = wid % nwin, z = (wid / nwin) % nz, ch = wid / (nwin * nz);
  const int l0 = ch * chunk;
  if (l0 >= ny) return;  // the whole wave
  const int l1 = min(l0 + chunk, ny);
  const int x0 = win * usew, nout = min(usew, nx - x0);  // the window's outputs x0 .. x0 + nout - 1
  const int wl = min(2 * lane, nout + 2 * HL - 2);        // window node of the lane's pair
  const unsigned vx = 4u * unsigned(wrapk(x0 - HL + wl, nx));
  const bool lane_out = 2 * lane >= HL && 2 * lane < HL + nout;
  const unsigned rowb = 4u * unsigned(nx);
  const unsigned zoff = unsigned(z) * unsigned(ny) * rowb;
  auto wrapped = [&](int m) {
    m %= ny;
    return m < 0 ? m + ny : m;
  };
  const int m0 = l0 - 3 * R, m1 = l1 + 3 * R;  // steps m0 .. m1 - 1
  // loads run PD steps ahead: K, or K/2 at reach 3 (60 registers fewer,
  // still thousands of cycles ahead at that kernel's occupancy)
  constexpr int PD = R == 3 ? K / 2 : K;
  static_assert(K % PD == 0, "prefetch slots are ring indices mod PD");
  float pr[2][K], p1[2][K], er[2][K], cr[2][K];  // rings, per node of the pair
  float np[2][PD], nc[2][PD], nu[2][PD];         // loads of the next PD steps (nu: x velocity)
  int lrow = wrapped(m0);                         // row of the next phi / y-velocity load
  int xrow = XFIRST ? lrow : wrapped(m0 - 3 * R); // row of the next x-velocity load
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int v = 0; v < 2; ++v) pr[v][i] = p1[v][i] = er[v][i] = cr[v][i] = 0.f;
#pragma unroll
  for (int i = 0; i < PD; ++i) {
    const unsigned ro = zoff + unsigned(lrow) * rowb;
    ld2_row(phi, vx, ro, np[0][i], np[1][i]);
    ld2_row(uy, vx, ro, nc[0][i], nc[1][i]);
    ld2_row(ux, vx, zoff + unsigned(xrow) * rowb, nu[0][i], nu[1][i]);
    lrow = lrow + 1 == ny ? 0 : lrow + 1;
    xrow = xrow + 1 == ny ? 0 : xrow + 1;
    __builtin_amdgcn_sched_barrier(0);  // in step order, as in k_sweep_m
  }
  int srow = wrapped(m0 - 3 * R);  // row of node m - 3R
  bool over = false;
  for (int mb = m0; mb < m1; mb += K) {
    static_for<K>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const int m = mb + i;
      // x Courant numbers of row m (XFIRST) or of row m - 3R
      constexpr int q = i % PD;  // prefetch slot of this step
      const float cxa = opaque(nu[0][q]) * lamx, cxb = opaque(nu[1][q]) * lamx;
      {
        float a = opaque(np[0][q]), b = opaque(np[1][q]);
        if (XFIRST) xsweep_pair<R, COMB>(a, b, cxa, cxb, over);
        pr[0][i] = a;
        pr[1][i] = b;
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) cr[v][i] = opaque(nc[v][q]) * lamy;
      {  // unconditional, all K steps, as in k_sweep_m
        const unsigned rn = zoff + unsigned(lrow) * rowb;
        ld2_row(phi, vx, rn, np[0][q], np[1][q]);
        ld2_row(uy, vx, rn, nc[0][q], nc[1][q]);
        ld2_row(ux, vx, zoff + unsigned(xrow) * rowb, nu[0][q], nu[1][q]);
      }
      lrow = lrow + 1 == ny ? 0 : lrow + 1;
      xrow = xrow + 1 == ny ? 0 : xrow + 1;
      constexpr int j1 = pmod(i - R, K), j2 = pmod(i - 2 * R, K), j3 = pmod(i - 3 * R, K);
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        {  // Phi1 of node m - R
          const DepN d = depart_n<R>(cr[v][j1], over);
          float a, b;
          ring_pair<R, K, j1>(pr[v], d, a, b);
          p1[v][j1] = lerp(a, b, d.f);
        }
        {  // e of node m - 2R
          const DepN d = depart_n<R>(-cr[v][j2], over);
          float a, b;
          ring_pair<R, K, j2>(p1[v], d, a, b);
          er[v][j2] = pr[v][j2] - lerp(a, b, d.f);
        }
      }
      // out of node m - 3R
      if (m - 3 * R >= l0 && m - 3 * R < l1) {
        float o[2];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const DepN d = depart_n<R>(cr[v][j3], over);
          float ea, eb;
          ring_pair<R, K, j3>(er[v], d, ea, eb);
          o[v] = sweep_combine<COMB>(p1[v][j3], er[v][j3], ea, eb, d.f);
        }
        if (!XFIRST) xsweep_pair<R, COMB>(o[0], o[1], cxa, cxb, over);
        if (lane_out) st2_row(out, vx, zoff + unsigned(srow) * rowb, o[0], o[1]);
      }
      srow = srow + 1 == ny ? 0 : srow + 1;
    });
  }
  if (over) *flag = 1;
}

template <typename F>
hipError_t set_lds(F kernel, int bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int NDIM, int SCHEME, int R>
hipError_t launch_ec_t(const Geo& g, const float* phi, const float* u, float* out, int* flag,
                       hipStream_t st) {
  constexpr int TX = R <= 2 ? 64 : 32;
  constexpr int TY = NDIM >= 2 ? 8 : 1;
  using S = EcShape<NDIM, SCHEME, R, TX, TY>;
  constexpr int bytes = S::FLOATS * 4;
  static_assert(bytes <= 160 * 1024, "LDS budget");
  auto kern = k_ec<NDIM, SCHEME, R, TX, TY>;
  static hipError_t attr = set_lds(kern, bytes);
  if (attr != hipSuccess) return attr;
  const size_t n = (size_t)g.ncells;
  const float* ux = u;
  const float* uy = NDIM >= 2 ? u + n : u;
  const float* uz = NDIM == 3 ? u + 2 * n : u;
  const int zchunk = NDIM == 3 ? 32 : 1;
  dim3 grid((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, (g.nz + zchunk - 1) / zchunk);
  hipLaunchKernelGGL(kern, grid, dim3(kThreads), bytes, st, phi, ux, uy, uz, out, g, zchunk, flag);
  return hipGetLastError();
}

template <int NDIM, int SCHEME>
hipError_t launch_ec_r(int R, const Geo& g, const float* phi, const float* u, float* out,
                       int* flag, hipStream_t st) {
  switch (R) {
    case 1: return launch_ec_t<NDIM, SCHEME, 1>(g, phi, u, out, flag, st);
    case 2: return launch_ec_t<NDIM, SCHEME, 2>(g, phi, u, out, flag, st);
    case 3: return launch_ec_t<NDIM, SCHEME, 3>(g, phi, u, out, flag, st);
    case 4: return launch_ec_t<NDIM, SCHEME, 4>(g, phi, u, out, flag, st);
  }
  return hipErrorInvalidValue;
}

template <int R, int COMB = kCombCec>
hipError_t launch_sweep_t(int d, const Geo& g, const float* phi, const float* ud, float* out,
                          int* flag, hipStream_t st, bool march) {
  if (d != 0 && march && offsets32_ok(g)) {
    const int L = d == 1 ? g.ny : g.nz;
    const int other = d == 1 ? g.nz : g.ny;
    const unsigned S4 = 4u * unsigned(d == 1 ? g.nx : g.nx * g.ny);
    const unsigned So4 = 4u * unsigned(d == 1 ? g.nx * g.ny : g.nx);
    // two columns per lane with an even nx up to reach 3 (at reach 4 the
    // rings would cost occupancy); enough waves to fill the chip (about 8
    // per CU), chunks of >= 16R nodes
    const bool two = g.nx % 2 == 0 && R <= 3;
    const int cols = two ? 128 : 64;
    const long long waves = (long long)((g.nx + cols - 1) / cols) * other;
    const int want = int(std::min<long long>((2048 + waves - 1) / waves, std::max(1, L / (16 * R))));
    const int chunk = (L + want - 1) / want;
    dim3 grid((g.nx + cols - 1) / cols, (other + 3) / 4, (L + chunk - 1) / chunk);
    if constexpr (R <= 3) {
      if (two) {
        hipLaunchKernelGGL((k_sweep_m<R, 2, COMB>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, L, S4,
                           So4, other, chunk, g.lam[d], flag);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_sweep_m<R, 1, COMB>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, L, S4,
                       So4, other, chunk, g.lam[d], flag);
    return hipGetLastError();
  }
  if (d == 0 && march && offsets32_ok(g)) {
    const int nrows = g.ny * g.nz;
    const int nwin = (g.nx + 64 - 6 * R - 1) / (64 - 6 * R);
    const long long waves = (long long)nrows * ((nwin + 3) / 4);
    hipLaunchKernelGGL((k_sweep_xw<R, COMB>), dim3(unsigned((waves + 3) / 4)), dim3(kThreads), 0, st, phi, ud,
                       out, g.nx, nrows, nwin, g.lam[0], flag);
    return hipGetLastError();
  }
  if (d == 0) {
    dim3 grid((g.nx + 255) / 256, (g.ny + 3) / 4, g.nz);
    hipLaunchKernelGGL((k_sweep_x<R, COMB>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, g.ny,
                       g.lam[0], flag);
  } else {
    const int L = d == 1 ? g.ny : g.nz;
    const int64_t S = d == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny;
    const int other = d == 1 ? g.nz : g.ny;
    const int64_t So = d == 1 ? (int64_t)g.nx * g.ny : (int64_t)g.nx;
    dim3 grid((g.nx + 63) / 64, (L + 31) / 32, other);
    hipLaunchKernelGGL((k_sweep_s<R, COMB>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, L, S, So,
                       g.lam[d], flag);
  }
  return hipGetLastError();
}

}  // namespace

namespace {
constexpr int kGatherCpt = 4;  // nodes per thread of the gather kernels
template <int MODE>
hipError_t launch_gather_m(int ndim, const Geo& g, const float* a, const float* b, const float* u,
                           float* out, int* flag, hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  const float* ux = u;
  const float* uy = ndim >= 2 ? u + n : u;
  const float* uz = ndim == 3 ? u + 2 * n : u;
  dim3 block(64, 4);
  dim3 grid((g.nx + 63) / 64, (g.ny + 4 * kGatherCpt - 1) / (4 * kGatherCpt), g.nz);
  switch (ndim) {
    case 1:
      hipLaunchKernelGGL((k_gather<1, MODE, kGatherCpt>), grid, block, 0, st, a, b, ux, uy, uz, out, g, flag);
      break;
    case 2:
      hipLaunchKernelGGL((k_gather<2, MODE, kGatherCpt>), grid, block, 0, st, a, b, ux, uy, uz, out, g, flag);
      break;
    case 3:
      hipLaunchKernelGGL((k_gather<3, MODE, kGatherCpt>), grid, block, 0, st, a, b, ux, uy, uz, out, g, flag);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_cir(int ndim, const Geo& g, const float* phi, const float* u, float* out,
                      int* flag, hipStream_t st) {
  return launch_gather_m<0>(ndim, g, phi, phi, u, out, flag, st);
}

hipError_t launch_ec_gather(int ndim, int mode, const Geo& g, const float* a, const float* b,
                            const float* u, float* out, int* flag, hipStream_t st) {
  if (mode == 1) return launch_gather_m<1>(ndim, g, a, b, u, out, flag, st);
  if (mode == 2) return launch_gather_m<2>(ndim, g, a, b, u, out, flag, st);
  return hipErrorInvalidValue;
}

hipError_t launch_ec(int ndim, int scheme, int R, const Geo& g, const float* phi, const float* u,
                     float* out, int* flag, hipStream_t st) {
  if (scheme == FEC) {
    switch (ndim) {
      case 1: return launch_ec_r<1, FEC>(R, g, phi, u, out, flag, st);
      case 2: return launch_ec_r<2, FEC>(R, g, phi, u, out, flag, st);
      case 3: return launch_ec_r<3, FEC>(R, g, phi, u, out, flag, st);
    }
  } else if (scheme == BEC) {
    switch (ndim) {
      case 1: return launch_ec_r<1, BEC>(R, g, phi, u, out, flag, st);
      case 2: return launch_ec_r<2, BEC>(R, g, phi, u, out, flag, st);
      case 3: return launch_ec_r<3, BEC>(R, g, phi, u, out, flag, st);
    }
  }
  return hipErrorInvalidValue;
}

template <int R, int COMB>
hipError_t launch_sweep_xy_t(bool xfirst, const Geo& g, const float* phi, const float* u,
                             float* out, int* flag, hipStream_t st) {
  constexpr int USE = 64 - 6 * R;
  const size_t n = (size_t)g.ncells;
  const int nwin = (g.nx + USE - 1) / USE;
  // chunks along y: about 8192 waves for the chip, chunks of >= 16R rows
  const long long per = (long long)nwin * g.nz;
  const int want = int(std::min<long long>((8192 + per - 1) / per, std::max(1, g.ny / (16 * R))));
  const int chunk = (g.ny + want - 1) / want;
  const long long waves = per * ((g.ny + chunk - 1) / chunk);
  const dim3 grid(unsigned((waves + 3) / 4));
  if (xfirst)
    hipLaunchKernelGGL((k_sweep_xym<R, true, COMB>), grid, dim3(kThreads), 0, st, phi, u, u + n, out, g.nx,
                       g.ny, g.nz, nwin, chunk, g.lam[0], g.lam[1], flag);
  else
    hipLaunchKernelGGL((k_sweep_xym<R, false, COMB>), grid, dim3(kThreads), 0, st, phi, u, u + n, out,
                       g.nx, g.ny, g.nz, nwin, chunk, g.lam[0], g.lam[1], flag);
  return hipGetLastError();
}

// Waves a launch of k_sweep_xyp aims for at reach 1 and 2 (32 per CU;
// half as many at reach 3, whose chunks carry 18 halo rows): its chunks
// along y are the longest that still give that many, and at least 16R rows.
// Measured at 512^3: 4096 and 16384 are 2-3% slower at reach 2; 8192 is
// 1% slower than 4096 at reach 3.
#ifndef SLA_XYP_WAVES
#define SLA_XYP_WAVES 8192
#endif

template <int R, int COMB>
hipError_t launch_sweep_xyp_t(bool xfirst, const Geo& g, const float* phi, const float* u,
                              float* out, int* flag, hipStream_t st) {
  constexpr int USE = 128 - 2 * pair_halo<R>();  // most outputs of a window
  const size_t n = (size_t)g.ncells;
  // balanced windows: usew outputs each (even), every window non-empty
  int nwin = (g.nx + USE - 1) / USE;
  int usew = (g.nx + nwin - 1) / nwin;
  usew += usew & 1;
  nwin = (g.nx + usew - 1) / usew;
  const long long per = (long long)nwin * g.nz;
  constexpr long long target = R >= 3 ? SLA_XYP_WAVES / 2 : SLA_XYP_WAVES;
  const int want = int(std::min<long long>((target + per - 1) / per, std::max(1, g.ny / (16 * R))));
  const int chunk = (g.ny + want - 1) / want;
  const long long waves = per * ((g.ny + chunk - 1) / chunk);
  const dim3 grid(unsigned((waves + 3) / 4));
  if (xfirst)
    hipLaunchKernelGGL((k_sweep_xyp<R, true, COMB>), grid, dim3(kThreads), 0, st, phi, u, u + n, out, g.nx,
                       g.ny, g.nz, nwin, usew, chunk, g.lam[0], g.lam[1], flag);
  else
    hipLaunchKernelGGL((k_sweep_xyp<R, false, COMB>), grid, dim3(kThreads), 0, st, phi, u, u + n, out,
                       g.nx, g.ny, g.nz, nwin, usew, chunk, g.lam[0], g.lam[1], flag);
  return hipGetLastError();
}

namespace {
template <int COMB>
hipError_t launch_sweep_xy_c(int R, bool xfirst, const Geo& g, const float* phi, const float* u,
                             float* out, int* flag, hipStream_t st, bool pairs) {
  if (!offsets32_ok(g)) return hipErrorInvalidValue;
  if (pairs) {
    if (g.nx % 2 != 0) return hipErrorInvalidValue;
    switch (R) {
      case 1: return launch_sweep_xyp_t<1, COMB>(xfirst, g, phi, u, out, flag, st);
      case 2: return launch_sweep_xyp_t<2, COMB>(xfirst, g, phi, u, out, flag, st);
      case 3: return launch_sweep_xyp_t<3, COMB>(xfirst, g, phi, u, out, flag, st);
    }
    return hipErrorInvalidValue;
  }
  switch (R) {  // one node per lane: reach 3 and more run one sweep per axis (see the caller)
    case 1: return launch_sweep_xy_t<1, COMB>(xfirst, g, phi, u, out, flag, st);
    case 2: return launch_sweep_xy_t<2, COMB>(xfirst, g, phi, u, out, flag, st);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_cec_sweep_xy(int R, bool xfirst, const Geo& g, const float* phi, const float* u,
                               float* out, int* flag, hipStream_t st, bool pairs, int scheme) {
  switch (scheme) {
    case CEC: return launch_sweep_xy_c<kCombCec>(R, xfirst, g, phi, u, out, flag, st, pairs);
    case FEC: return launch_sweep_xy_c<kCombFec>(R, xfirst, g, phi, u, out, flag, st, pairs);
    case BEC: return launch_sweep_xy_c<kCombBec>(R, xfirst, g, phi, u, out, flag, st, pairs);
    case CEC_LITERAL: return launch_sweep_xy_c<kCombCecLit>(R, xfirst, g, phi, u, out, flag, st, pairs);
  }
  return hipErrorInvalidValue;
}

namespace {
template <int R, int COMB, bool MID = false>
hipError_t launch_split_t(int d, const Geo& g, const float* phi, const float* ud, float* out,
                          int* flag, hipStream_t st) {
  if (d == 0) {
    dim3 grid((g.nx + 255) / 256, (g.ny + 3) / 4, g.nz);
    hipLaunchKernelGGL((k_sweep_x<R, COMB, MID>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, g.ny,
                       g.lam[0], flag);
  } else {
    const int L = d == 1 ? g.ny : g.nz;
    const int64_t S = d == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny;
    const int other = d == 1 ? g.nz : g.ny;
    const int64_t So = d == 1 ? (int64_t)g.nx * g.ny : (int64_t)g.nx;
    dim3 grid((g.nx + 63) / 64, (L + 31) / 32, other);
    hipLaunchKernelGGL((k_sweep_s<R, COMB, MID>), grid, dim3(kThreads), 0, st, phi, ud, out, g.nx, L, S,
                       So, g.lam[d], flag);
  }
  return hipGetLastError();
}
template <int COMB, bool MID = false>
hipError_t launch_split_r(int d, int R, const Geo& g, const float* phi, const float* ud, float* out,
                          int* flag, hipStream_t st) {
  switch (R) {
    case 1: return launch_split_t<1, COMB, MID>(d, g, phi, ud, out, flag, st);
    case 2: return launch_split_t<2, COMB, MID>(d, g, phi, ud, out, flag, st);
    case 3: return launch_split_t<3, COMB, MID>(d, g, phi, ud, out, flag, st);
    case 4: return launch_split_t<4, COMB, MID>(d, g, phi, ud, out, flag, st);
  }
  return hipErrorInvalidValue;
}
}  // namespace

namespace {
template <int COMB>
hipError_t launch_sweep_c(int d, int R, const Geo& g, const float* phi, const float* ud, float* out,
                          int* flag, hipStream_t st, bool march) {
  switch (R) {
    case 1: return launch_sweep_t<1, COMB>(d, g, phi, ud, out, flag, st, march);
    case 2: return launch_sweep_t<2, COMB>(d, g, phi, ud, out, flag, st, march);
    case 3: return launch_sweep_t<3, COMB>(d, g, phi, ud, out, flag, st, march);
    case 4: return launch_sweep_t<4, COMB>(d, g, phi, ud, out, flag, st, march);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_ec_sweep(int scheme, int d, int R, const Geo& g, const float* phi,
                           const float* ud, float* out, int* flag, hipStream_t st, bool march) {
  if (scheme == FEC) return launch_sweep_c<kCombFec>(d, R, g, phi, ud, out, flag, st, march);
  if (scheme == BEC) return launch_sweep_c<kCombBec>(d, R, g, phi, ud, out, flag, st, march);
  if (scheme == CEC_LITERAL) return launch_sweep_c<kCombCecLit>(d, R, g, phi, ud, out, flag, st, march);
  return hipErrorInvalidValue;
}

hipError_t launch_cec_sweep_mid(int d, int R, const Geo& g, const float* phi, const float* ud,
                                float* out, int* flag, hipStream_t st) {
  return launch_split_r<kCombCec, true>(d, R, g, phi, ud, out, flag, st);
}

hipError_t launch_cec_sweep(int d, int R, const Geo& g, const float* phi, const float* ud,
                            float* out, int* flag, hipStream_t st, bool march) {
  return launch_sweep_c<kCombCec>(d, R, g, phi, ud, out, flag, st, march);
}

}  // namespace sla
