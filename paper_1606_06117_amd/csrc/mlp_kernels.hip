// Learned per-cell correction: a 30->64->64->1 ReLU network run on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation), its training (forward, backward, Adam) and the fused
// inference step.
//
// Features of node i (32 inputs, the last two zero): the 27 differences
// Phi1[i+o] - Phi1[i] over the 3x3x3 neighbourhood (z outermost, x
// innermost) divided by sigma = sqrt(sum d^2 / 27 + 1e-30), then the node's
// Courant numbers c_x, c_y, c_z.  The network predicts y; the corrected
// value is Phi1[i] + sigma * y.  Phi1 is the CIR step (section 3); the
// training target is (third-order step - Phi1) / sigma.
//
// MFMA operand layout (16x16x32, one wave): with g = lane / 16 and
// c = lane % 16, lane holds A[c][8g..8g+7], B[8g..8g+7][c] and, after the
// instruction, D[4g..4g+3][c].  Every layer is computed transposed
// (hidden x cells), so a lane's four results are four consecutive hidden
// units of one cell and land in a row-major LDS tile as one 8-byte store.

#include <algorithm>
#include <cstddef>

#include "common.h"

namespace sla {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));
typedef unsigned uintx2 __attribute__((ext_vector_type(2)));

// Two values rounded to BF16 (to nearest, ties to even) in one register, lo
// in bits 0-15: written this way the pair becomes one conversion
// instruction (element-wise insertion into a wider vector does not).
__device__ __forceinline__ unsigned cvt_pk_bf16(float lo, float hi) {
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(unsigned, v);
}
typedef short s16x2 __attribute__((ext_vector_type(2)));
// ReLU of two packed BF16 values: a signed 16-bit maximum with 0 of each bit
// pattern (negative values and -0 become +0).  On rounded values it equals
// rounding after ReLU for every non-NaN value.  The empty asm statement
// keeps the compiler from splitting the paired conversion that produced v
// into two single ones.
__device__ __forceinline__ unsigned relu_pk(unsigned v) {
  asm("" : "+v"(v));
  return __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{}));
}

// max(v, 0) as a signed integer maximum of the bit pattern with 0: negative
// values (sign bit set) and -0 become +0, the rest stay.  The same value as
// fmaxf(v, 0.f) for every non-NaN v, in one instruction (fmaxf also
// quiets a possible signalling NaN first, one more instruction).
__device__ __forceinline__ float relu_bits(float v) {
  return __builtin_bit_cast(float, max(__builtin_bit_cast(int, v), 0));
}

constexpr int kThreads = 256;
constexpr int NF = kMlpInputs, NH = kMlpHidden;
constexpr int W1_OFF = 0, B1_OFF = NF * NH, W2_OFF = B1_OFF + NH, B2_OFF = W2_OFF + NH * NH,
              W3_OFF = B2_OFF + NH, B3_OFF = W3_OFF + NH;
static_assert(B3_OFF + 1 == kMlpParams, "parameter layout");

__device__ __forceinline__ floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ void st4(__bf16* p, float a, float b, float c, float d) {
  bf16x4 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  v[2] = (__bf16)c;
  v[3] = (__bf16)d;
  *reinterpret_cast<bf16x4*>(p) = v;
}

// sum over the 16 lanes that share g (lane bits 0..3), by DPP within the
// 16-lane row (no LDS): swap neighbours, swap pairs, mirror the half rows,
// mirror the row.  Each step adds two sums that every lane forms in the
// same order, so all 16 lanes end with the same value.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float sum16(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_f<0x141>(v);  // row_half_mirror: quads 0-1 and 2-3 swap
  v += dpp_f<0x140>(v);  // row_mirror: the 8-lane halves swap
  return v;
}
// sum over the 4 lanes that share c (lane bits 4..5)
__device__ __forceinline__ float sum4g(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ float min4g(float v) {
  v = fminf(v, __shfl_xor(v, 16));
  return fminf(v, __shfl_xor(v, 32));
}
__device__ __forceinline__ float max4g(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  return fmaxf(v, __shfl_xor(v, 32));
}

// LDS row strides (BF16 elements), padded by 16 bytes: a matrix-core
// operand read takes 16 bytes from each of 16 rows, and with rows 64 or 128
// bytes apart those rows would share banks; 80 and 144 bytes spread every 8
// consecutive rows over all 32 banks.
constexpr int SF = NF + 8;  // rows of 32 (W1T rows; [feature|hidden][cell] tiles)
constexpr int SH = NH + 8;  // rows of 64 (W2T, W2R, [cell][hidden] tiles)
constexpr int SC = 32 + 8;  // rows of 32 cells

// Weights in LDS: W1T [n][k] (64 x 32), W2T [n][k] (64 x 64), all BF16 with
// padded rows; biases and w3 FP32 (already BF16-rounded).  Training also
// keeps W2R [k][n] (64 x 64).
struct alignas(16) WeightsLds {
  __bf16 w1t[NH * SF];
  __bf16 w2t[NH * SH];
  float b1[NH], b2[NH], w3[NH], b3;
};
// the biases are read four at a time as MFMA accumulator seeds
static_assert(offsetof(WeightsLds, b1) % 16 == 0 && offsetof(WeightsLds, b2) % 16 == 0,
              "bias rows must be 16-byte aligned");

__device__ void load_weights(WeightsLds& W, __bf16* w2r, const __bf16* __restrict__ wpack,
                             const float* __restrict__ wr) {
  for (int i = threadIdx.x; i < NH * NF; i += kThreads) W.w1t[(i / NF) * SF + i % NF] = wpack[i];
  for (int i = threadIdx.x; i < NH * NH; i += kThreads)
    W.w2t[(i / NH) * SH + i % NH] = wpack[NH * NF + i];
  if (w2r)
    for (int i = threadIdx.x; i < NH * NH; i += kThreads)
      w2r[(i / NH) * SH + i % NH] = wpack[NH * NF + NH * NH + i];
  for (int i = threadIdx.x; i < NH; i += kThreads) {
    W.b1[i] = wr[B1_OFF + i];
    W.b2[i] = wr[B2_OFF + i];
    W.w3[i] = wr[W3_OFF + i];
  }
  if (threadIdx.x == 0) W.b3 = wr[B3_OFF];
}

// Order a wave's LDS writes before its later LDS reads of what other lanes of
// the same wave wrote (and reads before later rewrites).  The tiles in LDS
// belong to one wave each, so no workgroup barrier is needed: the waves of a
// workgroup run their tiles independently.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward pass of one 32-cell tile held by one wave.  xb[jt] is the B
// operand of cells 16 jt + c (features 8g..8g+7).  Writes H1 (row-major
// [cell][hidden], BF16) to h1, returns h2 (transposed tiles, FP32, after the
// ReLU) in h2 and y of cell 16 jt + c (on every lane of that cell).
__device__ __forceinline__ void forward_tile(const WeightsLds& W, const bf16x8 xb[2], __bf16* h1,
                                             floatx4 h2[4][2], float y[2]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  // layer 1: H1T[k][j] = sum_i W1T[k][i] X[j][i]
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const bf16x8 a = ld8(&W.w1t[(16 * it + c) * SF + 8 * g]);
    const int k = 16 * it + 4 * g;
    const floatx4 bias = *reinterpret_cast<const floatx4*>(&W.b1[k]);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      // the bias starts the accumulation (one vector add fewer per output)
      const floatx4 acc = mfma(a, xb[jt], bias);
      st4(&h1[(16 * jt + c) * SH + k], fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f),
          fmaxf(acc[3], 0.f));
    }
  }
  wave_lds_sync();
  // layer 2: H2T[n][j] = sum_k W2T[n][k] H1[j][k], two K steps of 32
  float s[2] = {0.f, 0.f};
#pragma unroll
  for (int it = 0; it < 4; ++it) {
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int n = 16 * it + 4 * g;
      floatx4 acc = *reinterpret_cast<const floatx4*>(&W.b2[n]);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
        acc = mfma(ld8(&W.w2t[(16 * it + c) * SH + 32 * kk + 8 * g]),
                   ld8(&h1[(16 * jt + c) * SH + 32 * kk + 8 * g]), acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[q] = fmaxf(acc[q], 0.f);
        s[jt] = fmaf(acc[q], W.w3[n + q], s[jt]);
      }
      h2[it][jt] = acc;
    }
  }
  wave_lds_sync();  // h1 is rewritten by the wave's next tile
  // layer 3: y = h2 . w3 + b3, summed over the 4 lanes holding the cell
  y[0] = sum4g(s[0]) + W.b3;
  y[1] = sum4g(s[1]) + W.b3;
}

// ---------------------------------------------------------------------------
// Evaluation on feature rows: X holds m rows of 32 BF16 features; y of every
// row to yout.  Every wave of a block runs the same number of tiles.
// ---------------------------------------------------------------------------
struct EvalLds {
  WeightsLds W;
  __bf16 h1[4][32 * SH];  // [cell][hidden]
};

__global__ __launch_bounds__(kThreads) void k_mlp_eval(const __bf16* __restrict__ X, int m,
                                                       int tiles_per_wave,
                                                       const __bf16* __restrict__ wpack,
                                                       const float* __restrict__ wr,
                                                       float* __restrict__ yout) {
  __shared__ __align__(16) EvalLds L;
  load_weights(L.W, nullptr, wpack, wr);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, w = threadIdx.x >> 6;
  for (int tt = 0; tt < tiles_per_wave; ++tt) {
    const int r0 = ((blockIdx.x * tiles_per_wave + tt) * 4 + w) * 32;
    bf16x8 xb[2];
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int row = r0 + 16 * jt + c;
      if (row < m) {
        xb[jt] = ld8(&X[(size_t)row * NF + 8 * g]);
      } else {
#pragma unroll
        for (int v = 0; v < 8; ++v) xb[jt][v] = (__bf16)0.f;
      }
    }
    floatx4 h2[4][2];
    float y[2];
    forward_tile(L.W, xb, L.h1[w], h2, y);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int row = r0 + 16 * jt + c;
      if (g == 0 && row < m) yout[row] = y[jt];
    }
  }
}

// ---------------------------------------------------------------------------
// Training on feature rows: the gradient of mean((y - t)^2) (inv_m2 =
// 2 / m_total) summed over the block's rows into gpart[blockIdx]
// [kMlpPartStride] (in the partial order below) and the squared error into
// lpart[blockIdx].  A wave runs 32-row tiles;
// every product of the backward pass is a matrix-core product.  Those whose
// reduction runs over the tile's rows (the weight gradients) take both
// operands with the rows as the K index: each operand is kept in LDS as a
// row-major [row][unit] tile, written with one vector store per lane from
// the layout the forward pass produced, and read into the operand layout by
// gfx950's transposing LDS load (ds_read_b64_tr_b16: within 16 lanes, lane r
// gives the address of 4 consecutive 16-bit values and receives value q
// from lane r/4 + 4q, element r%4).  The tiles belong to one wave: a
// wave-scope LDS fence orders them, no workgroup barrier.  The waves' sums
// are added in a fixed order at the end (deterministic).
// ---------------------------------------------------------------------------
// Order of a training block's gradient partials (and of the slots they are
// summed in): four values of a lane together, then the next lane: value v
// of lane l (l = 16 g + c) at (v / 4) * 256 + 4 l + v % 4, so a lane writes
// an MFMA tile's four results with one 16-byte store and a store of the
// wave covers 1 KB without a bank conflict.  Values 0..63 are the W2 tiles,
// (nt * 4 + kt) * 4 + q for W2[16 kt + c][16 nt + 4 g + q]; 64..95 the W1
// tiles, 64 + (kt * 2 + it) * 4 + q for W1[16 it + c][16 kt + 4 g + q];
// then, from kPosUnits, w3, b2 and b1 by unit, b3, and the squared error.
constexpr int kPosW1 = 64 * 64, kPosUnits = 96 * 64, kPosLoss = kPosUnits + 193;
static_assert(kPosLoss == kMlpParams, "one position per parameter, then the loss");
__device__ __forceinline__ int param_of_pos(int pos) {
  if (pos < kPosUnits) {
    const int v = (pos / 256) * 4 + pos % 4, l = (pos / 4) % 64;
    if (v < 64)
      return W2_OFF + (16 * ((v / 4) % 4) + l % 16) * NH + 16 * (v / 16) + 4 * (l / 16) + v % 4;
    const int u = v - 64;
    return W1_OFF + (16 * ((u / 4) % 2) + l % 16) * NH + 16 * (u / 8) + 4 * (l / 16) + u % 4;
  }
  const int j = pos - kPosUnits;
  return j < 64 ? W3_OFF + j : j < 128 ? B2_OFF + (j - 64) : j < 192 ? B1_OFF + (j - 128) : B3_OFF;
}

constexpr int kTrWaves = 8;
struct TrainLds {
  WeightsLds W;
  alignas(16) __bf16 w2r[NH * SH];  // W2R [k][n]
  union alignas(16) {
    struct {
      __bf16 x[kTrWaves][32 * SF];    // [row][feature]
      __bf16 h1[kTrWaves][32 * SH];   // [row][hidden]
      __bf16 dh2[kTrWaves][32 * SH];  // [row][n]
      __bf16 dh1[kTrWaves][32 * SH];  // [row][k]
    } t;
    float red[4][kMlpPartStride];  // the waves' sums, four slots in partial order
  } u;
};

// Operands of products whose K index is the tile's 32 rows, from a
// row-major tile T (row stride S BF16 values): operand t of NOPS receives
// at lane (g, c) T[8g .. 8g+7][16 t + c], the A operand of rows 16t..16t+15
// of the product's left factor, or the B operand of its columns
// 16t..16t+15.  Lane (g, r) addresses row 8g + r/4, columns 4 (r%4) ..
// +3 of each 16-column block, for rows 8g..8g+3 and again 4 rows down.
// The reads are written in assembly: the compiler's builtin for this
// instruction returns each lane's four values as copies of the first.  The
// block waits for its own reads, so no load is left in flight.
template <int S, int NOPS>
__device__ __forceinline__ void ld_rows_ops(const __bf16* T, int lane, bf16x8 (&o)[NOPS]) {
  static_assert(NOPS == 2 || NOPS == 4, "two or four 16-column blocks");
  const int g = lane >> 4, r = lane & 15;
  typedef __attribute__((address_space(3))) const __bf16 lds_bf16;
  const unsigned a = unsigned(reinterpret_cast<size_t>((lds_bf16*)(T + (8 * g + r / 4) * S + 4 * (r % 4))));
  uintx2 v[8];
  if constexpr (NOPS == 4) {
    asm volatile(
        "ds_read_b64_tr_b16 %0, %8\n\t"
        "ds_read_b64_tr_b16 %1, %8 offset:%9\n\t"
        "ds_read_b64_tr_b16 %2, %8 offset:32\n\t"
        "ds_read_b64_tr_b16 %3, %8 offset:%10\n\t"
        "ds_read_b64_tr_b16 %4, %8 offset:64\n\t"
        "ds_read_b64_tr_b16 %5, %8 offset:%11\n\t"
        "ds_read_b64_tr_b16 %6, %8 offset:96\n\t"
        "ds_read_b64_tr_b16 %7, %8 offset:%12\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]), "=&v"(v[6]),
          "=&v"(v[7])
        : "v"(a), "i"(8 * S), "i"(8 * S + 32), "i"(8 * S + 64), "i"(8 * S + 96)
        : "memory");
  } else {
    asm volatile(
        "ds_read_b64_tr_b16 %0, %4\n\t"
        "ds_read_b64_tr_b16 %1, %4 offset:%5\n\t"
        "ds_read_b64_tr_b16 %2, %4 offset:32\n\t"
        "ds_read_b64_tr_b16 %3, %4 offset:%6\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3])
        : "v"(a), "i"(8 * S), "i"(8 * S + 32)
        : "memory");
  }
#pragma unroll
  for (int t = 0; t < NOPS; ++t)
    o[t] = __builtin_bit_cast(bf16x8, uintx4{v[2 * t][0], v[2 * t][1], v[2 * t + 1][0], v[2 * t + 1][1]});
}

__global__ __launch_bounds__(64 * kTrWaves) void k_mlp_train(const __bf16* __restrict__ X,
                                                             const float* __restrict__ target,
                                                             int m, float inv_m2, int tiles_per_wave,
                                                             const __bf16* __restrict__ wpack,
                                                             const float* __restrict__ wr,
                                                             float* __restrict__ gpart,
                                                             float* __restrict__ lpart) {
  extern __shared__ __align__(16) unsigned char smem[];
  TrainLds& L = *reinterpret_cast<TrainLds*>(smem);
  constexpr int NT = 64 * kTrWaves;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, w = threadIdx.x >> 6;
  // rows of tile tt: B operands of the forward's first layer (features
  // 8g..8g+7 of rows 16 jt + c), loaded from a clamped row and zeroed past m
  // (no load under a condition)
  // (and their targets, 0 past m)
  auto load_x = [&](int tt, bf16x8 (&xb)[2], float (&tg)[2]) {
    const int r0 = ((blockIdx.x * tiles_per_wave + tt) * kTrWaves + w) * 32;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int row = r0 + 16 * jt + c;
      const uintx4 v = __builtin_bit_cast(uintx4, ld8(&X[(size_t)min(row, m - 1) * NF + 8 * g]));
      const float t = target[min(row, m - 1)];
      const unsigned keep = row < m ? ~0u : 0u;
      xb[jt] = __builtin_bit_cast(bf16x8, uintx4{v[0] & keep, v[1] & keep, v[2] & keep, v[3] & keep});
      tg[jt] = row < m ? t : 0.f;
    }
  };
  bf16x8 xnext[2];
  float tnext[2];
  load_x(0, xnext, tnext);  // in flight while the weights are staged
  // weights: 16-byte loads of the packed operand layouts into padded rows
  for (int i = threadIdx.x; i < NH * NF / 8; i += NT)
    *reinterpret_cast<bf16x8*>(&L.W.w1t[(i / (NF / 8)) * SF + 8 * (i % (NF / 8))]) = ld8(&wpack[8 * i]);
  for (int i = threadIdx.x; i < NH * NH / 8; i += NT) {
    const int row = i / (NH / 8), col = 8 * (i % (NH / 8));
    *reinterpret_cast<bf16x8*>(&L.W.w2t[row * SH + col]) = ld8(&wpack[NH * NF + 8 * i]);
    *reinterpret_cast<bf16x8*>(&L.w2r[row * SH + col]) = ld8(&wpack[NH * NF + NH * NH + 8 * i]);
  }
  for (int i = threadIdx.x; i < NH; i += NT) {
    L.W.b1[i] = wr[B1_OFF + i];
    L.W.b2[i] = wr[B2_OFF + i];
    L.W.w3[i] = wr[W3_OFF + i];
  }
  if (threadIdx.x == 0) L.W.b3 = wr[B3_OFF];
  __syncthreads();
  __bf16* xs = L.u.t.x[w];
  __bf16* h1 = L.u.t.h1[w];
  __bf16* dh2 = L.u.t.dh2[w];
  __bf16* dh1 = L.u.t.dh1[w];

  floatx4 dw2[4][4], dw1[4][2];  // dW2T[n][k], dW1T[k][i] tiles (D layout)
  // w3, b2 and b1 gradients of unit 16 (c / 4) + 4 g + c % 4: each tile's
  // sums over its rows, reduced over the 16 lanes of a row at once
  float own_w3 = 0.f, own_b2 = 0.f, own_b1 = 0.f, db3 = 0.f, sq = 0.f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) dw2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 2; ++b) dw1[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  // add this row's sums of a 16-value set (index 4a + q) to the lane's own
  auto own_add = [&](float& own, float (&t)[4][4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float v = sum16(t[a][q]);
        own += c == 4 * a + q ? v : 0.f;
      }
  };

  for (int tt = 0; tt < tiles_per_wave; ++tt) {
    const int r0 = ((blockIdx.x * tiles_per_wave + tt) * kTrWaves + w) * 32;
    bf16x8 xb[2] = {xnext[0], xnext[1]};
    const float tg[2] = {tnext[0], tnext[1]};
    load_x(min(tt + 1, tiles_per_wave - 1), xnext, tnext);  // the next tile's rows
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) *reinterpret_cast<bf16x8*>(&xs[(16 * jt + c) * SF + 8 * g]) = xb[jt];
    // ---- forward (as forward_tile), keeping which H1 entries are positive
    unsigned h1pos = 0;  // bit 8 it + 4 jt + q: H1[16 jt + c][16 it + 4g + q] > 0
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const bf16x8 a = ld8(&L.W.w1t[(16 * it + c) * SF + 8 * g]);
      const int k = 16 * it + 4 * g;
      const floatx4 bias = *reinterpret_cast<const floatx4*>(&L.W.b1[k]);
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) {
        const floatx4 acc = mfma(a, xb[jt], bias);
        float hv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          hv[q] = fmaxf(acc[q], 0.f);
          if ((float)(__bf16)hv[q] > 0.f) h1pos |= 1u << (8 * it + 4 * jt + q);
        }
        st4(&h1[(16 * jt + c) * SH + k], hv[0], hv[1], hv[2], hv[3]);
      }
    }
    wave_lds_sync();
    floatx4 h2[4][2];
    float s[2] = {0.f, 0.f};
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) {
        const int n = 16 * it + 4 * g;
        floatx4 acc = *reinterpret_cast<const floatx4*>(&L.W.b2[n]);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
          acc = mfma(ld8(&L.W.w2t[(16 * it + c) * SH + 32 * kk + 8 * g]),
                     ld8(&h1[(16 * jt + c) * SH + 32 * kk + 8 * g]), acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q] = fmaxf(acc[q], 0.f);
          s[jt] = fmaf(acc[q], L.W.w3[n + q], s[jt]);
        }
        h2[it][jt] = acc;
      }
    }
    float dy[2];
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int row = r0 + 16 * jt + c;
      const float y = sum4g(s[jt]) + L.W.b3;
      const float err = row < m ? y - tg[jt] : 0.f;
      dy[jt] = err * inv_m2;
      if (g == 0) {
        sq = fmaf(err, err, sq);
        db3 += dy[jt];
      }
    }
    // ---- backward: dH2 = dy w3 where H2 > 0, as [row][n]
    {
      float t3[4][4], t2[4][4];
#pragma unroll
      for (int it = 0; it < 4; ++it) {
#pragma unroll
        for (int q = 0; q < 4; ++q) t3[it][q] = t2[it][q] = 0.f;
#pragma unroll
        for (int jt = 0; jt < 2; ++jt) {
          const int n = 16 * it + 4 * g;
          float d[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            t3[it][q] = fmaf(h2[it][jt][q], dy[jt], t3[it][q]);
            d[q] = h2[it][jt][q] > 0.f ? dy[jt] * L.W.w3[n + q] : 0.f;
            t2[it][q] += d[q];
          }
          st4(&dh2[(16 * jt + c) * SH + n], d[0], d[1], d[2], d[3]);
        }
      }
      own_add(own_w3, t3);
      own_add(own_b2, t2);
    }
    wave_lds_sync();
    // dW2T[n][k] += sum over rows of dH2[row][n] H1[row][k]
    {
      bf16x8 a[4], bk[4];
      ld_rows_ops<SH, 4>(dh2, lane, a);
      ld_rows_ops<SH, 4>(h1, lane, bk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) dw2[nt][kt] = mfma(a[nt], bk[kt], dw2[nt][kt]);
    }
    // dH1T[k][row] = sum_n W2R[k][n] dH2[row][n], where H1 > 0; stored as [row][k]
    {
      float t1[4][4];
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) t1[kt][q] = 0.f;
#pragma unroll
        for (int jt = 0; jt < 2; ++jt) {
          floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int nn = 0; nn < 2; ++nn)
            acc = mfma(ld8(&L.w2r[(16 * kt + c) * SH + 32 * nn + 8 * g]),
                       ld8(&dh2[(16 * jt + c) * SH + 32 * nn + 8 * g]), acc);
          float d[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            d[q] = (h1pos >> (8 * kt + 4 * jt + q)) & 1u ? acc[q] : 0.f;
            t1[kt][q] += d[q];
          }
          st4(&dh1[(16 * jt + c) * SH + 16 * kt + 4 * g], d[0], d[1], d[2], d[3]);
        }
      }
      own_add(own_b1, t1);
    }
    wave_lds_sync();
    // dW1T[k][i] += sum over rows of dH1[row][k] X[row][i]
    {
      bf16x8 a[4], bx[2];
      ld_rows_ops<SH, 4>(dh1, lane, a);
      ld_rows_ops<SF, 2>(xs, lane, bx);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int it = 0; it < 2; ++it) dw1[kt][it] = mfma(a[kt], bx[it], dw1[kt][it]);
    }
    wave_lds_sync();  // the tiles are rewritten by the wave's next tile
  }

  // ---- the block's sum, in partial order: waves 0-3 write slots 0-3, waves
  // 4-7 add theirs to slot w - 4, then every position is summed over the
  // slots in slot order (lane-major, so no two lanes of an access share a
  // bank)
  const float rb3 = sum16(sum4g(db3));
  const float rsq = sum16(sum4g(sq));
  __syncthreads();  // the tiles' LDS becomes the slots
  for (int phase = 0; phase < 2; ++phase) {
    if ((w >= 4) == (phase == 1)) {
      float* acc = L.u.red[w & 3];
      const bool first = phase == 0;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
          floatx4* p = reinterpret_cast<floatx4*>(&acc[(nt * 4 + kt) * 256 + 4 * lane]);
          *p = first ? dw2[nt][kt] : *p + dw2[nt][kt];
        }
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          floatx4* p = reinterpret_cast<floatx4*>(&acc[kPosW1 + (kt * 2 + it) * 256 + 4 * lane]);
          *p = first ? dw1[kt][it] : *p + dw1[kt][it];
        }
      {
        const int n = kPosUnits + 16 * (c / 4) + 4 * g + c % 4;  // this lane's unit
        acc[n] = first ? own_w3 : acc[n] + own_w3;
        acc[n + 64] = first ? own_b2 : acc[n + 64] + own_b2;
        acc[n + 128] = first ? own_b1 : acc[n + 128] + own_b1;
      }
      if (lane == 0) {
        acc[kPosUnits + 192] = first ? rb3 : acc[kPosUnits + 192] + rb3;
        acc[kPosLoss] = first ? rsq : acc[kPosLoss] + rsq;
      }
    }
    __syncthreads();
  }
  float* gp = gpart + (size_t)blockIdx.x * kMlpPartStride;
  for (int i = 4 * threadIdx.x; i < kPosUnits; i += 4 * NT) {
    const floatx4* r0 = reinterpret_cast<const floatx4*>(&L.u.red[0][i]);
    const floatx4* r1 = reinterpret_cast<const floatx4*>(&L.u.red[1][i]);
    const floatx4* r2 = reinterpret_cast<const floatx4*>(&L.u.red[2][i]);
    const floatx4* r3 = reinterpret_cast<const floatx4*>(&L.u.red[3][i]);
    *reinterpret_cast<floatx4*>(&gp[i]) = (*r0 + *r1) + (*r2 + *r3);
  }
  for (int i = kPosUnits + threadIdx.x; i <= kPosLoss; i += NT) {
    const float v = (L.u.red[0][i] + L.u.red[1][i]) + (L.u.red[2][i] + L.u.red[3][i]);
    if (i < kPosLoss)
      gp[i] = v;
    else
      lpart[blockIdx.x] = v;
  }
}

// Adam (Kingma & Ba) on master weight p with gradient gr; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.  Returns the new weight.
// One Adam update in registers: moments m, v and weight w of a parameter
// with gradient gr.
__device__ __forceinline__ void adam_step(float& m, float& v, float& w, float gr, float lr,
                                          float beta1, float beta2, float eps, float bc1, float bc2) {
  m = beta1 * m + (1.f - beta1) * gr;
  v = beta2 * v + (1.f - beta2) * gr * gr;
  w = w - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

// Round the FP32 master weights to BF16 (FP32 copy `wr`) and write the
// matrix-core operand layouts.
__device__ __forceinline__ void pack_one(int p, float v, float* __restrict__ wr,
                                         __bf16* __restrict__ wpack) {
  const __bf16 b = (__bf16)v;
  wr[p] = (float)b;
  if (p < B1_OFF) {
    const int k = p / NH, n = p % NH;  // W1[k][n]
    wpack[n * NF + k] = b;
  } else if (p >= W2_OFF && p < B2_OFF) {
    const int q = p - W2_OFF, k = q / NH, n = q % NH;  // W2[k][n]
    wpack[NH * NF + n * NH + k] = b;
    wpack[NH * NF + NH * NH + k * NH + n] = b;
  }
}

// Sum per-block partials in a fixed order (deterministic), position by
// position (the training blocks' partial order), into the gradient of the
// parameter at that position.  A workgroup takes 32 positions; its 8 row groups each sum every 8th partial in
// block order, and the 8 sums are added in group order.  Workgroup 0 also
// sums the loss partials: 256 fixed strided sums, then a fixed tree.
constexpr int kRedParams = 32, kRedParts = kThreads / kRedParams;
struct AdamArgs {
  float* master;
  float* mo;
  float* vo;
  float lr, beta1, beta2, eps, bc1, bc2;
  float* wr;
  __bf16* wpack;
};
template <bool ADAM>
__global__ __launch_bounds__(kThreads) void k_grad_reduce(const float* __restrict__ gpart,
                                                          const float* __restrict__ lpart,
                                                          int nblk, float* __restrict__ grad,
                                                          double* __restrict__ loss_sum,
                                                          AdamArgs ad) {
  __shared__ float part[kRedParts][kRedParams];
  __shared__ double lsum[kThreads];
  const int pl = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
  const int p = blockIdx.x * kRedParams + pl;
  const bool own = grp == 0 && p < kMlpParams;  // the thread that finishes position p
  // Adam state of the position's parameter, loaded with the partials
  // instead of after the workgroup's sum
  const int pp = own ? param_of_pos(p) : 0;
  float am = 0.f, av = 0.f, aw = 0.f;
  if (ADAM && own) {
    am = ad.mo[pp];
    av = ad.vo[pp];
    aw = ad.master[pp];
  }
  float s = 0.f;
  if (p < kMlpParams) {
    int b = grp;
    constexpr int kInFlight = 32;  // 256 partials: every load of a thread in flight at once
    for (; b + (kInFlight - 1) * kRedParts < nblk; b += kInFlight * kRedParts) {
      float v[kInFlight];
#pragma unroll
      for (int q = 0; q < kInFlight; ++q) v[q] = gpart[(size_t)(b + q * kRedParts) * kMlpPartStride + p];
#pragma unroll
      for (int q = 0; q < kInFlight; ++q) s += v[q];
    }
    for (; b < nblk; b += kRedParts) s += gpart[(size_t)b * kMlpPartStride + p];
  }
  part[grp][pl] = s;
  if (blockIdx.x == 0) {
    double l = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) l += lpart[b];
    lsum[threadIdx.x] = l;
  }
  __syncthreads();
  if (own) {  // p: a partial's position
    float t = part[0][pl];
#pragma unroll
    for (int q = 1; q < kRedParts; ++q) t += part[q][pl];
    grad[pp] = t;
    if (ADAM) {  // the training step's Adam update of this parameter
      adam_step(am, av, aw, t, ad.lr, ad.beta1, ad.beta2, ad.eps, ad.bc1, ad.bc2);
      ad.mo[pp] = am;
      ad.vo[pp] = av;
      ad.master[pp] = aw;
      pack_one(pp, aw, ad.wr, ad.wpack);
    }
  }
  if (blockIdx.x == 0) {
    for (int h = kThreads / 2; h > 0; h /= 2) {
      if (int(threadIdx.x) < h) lsum[threadIdx.x] += lsum[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss_sum = lsum[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_pack(const float* __restrict__ master,
                                                   float* __restrict__ wr,
                                                   __bf16* __restrict__ wpack) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p < kMlpParams) pack_one(p, master[p], wr, wpack);
}

// ---------------------------------------------------------------------------
// Features of one node for the lane that holds inputs 8g..8g+7, and the
// node's sigma.  Every lane of the node's group computes the same sigma.
// ---------------------------------------------------------------------------
struct NodeFeatures {
  bf16x8 x;
  float sigma;
  float centre;
  float lo, hi;  // range of the 27 values around the node
};

// Features of a node from its gathered values: val[v] is the neighbour
// k = 8g + v (k < 27) of this lane's group, c3 the node's three Courant
// numbers (used by group 3).
__device__ __forceinline__ NodeFeatures features_from(const float (&val)[8], float centre, int g,
                                                      float cx, float cy, float cz) {
  float d[8];
  float ss = 0.f, lo = centre, hi = centre;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    d[v] = 0.f;
    if (8 * g + v < 27) {
      lo = fminf(lo, val[v]);
      hi = fmaxf(hi, val[v]);
      d[v] = val[v] - centre;
      ss = fmaf(d[v], d[v], ss);
    }
  }
  ss = sum4g(ss);
  NodeFeatures f;
  f.sigma = sqrtf(ss / 27.f + 1e-30f);
  f.centre = centre;
  f.lo = min4g(lo);
  f.hi = max4g(hi);
  const float inv = 1.f / f.sigma;
#pragma unroll
  for (int v = 0; v < 8; ++v) f.x[v] = (__bf16)(d[v] * inv);
  if (g == 3) {  // inputs 27..29: Courant numbers, 30..31 zero
    f.x[3] = (__bf16)cx;
    f.x[4] = (__bf16)cy;
    f.x[5] = (__bf16)cz;
    f.x[6] = (__bf16)0.f;
    f.x[7] = (__bf16)0.f;
  }
  return f;
}

// Gather with periodic wrap on every axis (any node).
__device__ __forceinline__ NodeFeatures node_features(const float* __restrict__ phi1,
                                                      const float* __restrict__ ux,
                                                      const float* __restrict__ uy,
                                                      const float* __restrict__ uz, const Geo& geo,
                                                      int x, int y, int z, int g) {
  const int nx = geo.nx, ny = geo.ny, nz = geo.nz;
  const size_t plane = (size_t)nx * ny;
  const size_t ic = (size_t)z * plane + (size_t)y * nx + x;
  float val[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int k = 8 * g + v;
    val[v] = 0.f;
    if (k < 27) {
      const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
      int xx = x + dx, yy = y + dy, zz = z + dz;
      xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
      yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
      zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
      val[v] = phi1[(size_t)zz * plane + (size_t)yy * nx + xx];
    }
  }
  return features_from(val, phi1[ic], g, ux[ic] * geo.lam[0], uy[ic] * geo.lam[1],
                       uz[ic] * geo.lam[2]);
}

// Buffer access with a 32-bit byte offset from a descriptor in scalar
// registers, for the learned step's gather: fields of fewer than 2^30 cells
// (a descriptor's size tops out one byte short of 2^32, so at 2^30 cells it
// would clip the field's last element; such fields take node_features).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc field_rsrc(const float* base, size_t n) {
  const unsigned bytes = n >= (size_t(1) << 30) ? 0xFFFFFFFFu : unsigned(n) * 4u;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), short(0), int(bytes), 0x00020000);
}
__device__ __forceinline__ float ld_at(Rsrc r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// Training pairs: features of the listed nodes (linear indices) from the CIR
// field phi1, and the target (phi_next - phi1) / sigma.  One wave handles 16
// nodes (4 lanes per node).
__global__ __launch_bounds__(kThreads) void k_make_pairs(const float* __restrict__ phi1,
                                                         const float* __restrict__ phi_next,
                                                         const float* __restrict__ ux,
                                                         const float* __restrict__ uy,
                                                         const float* __restrict__ uz, Geo geo,
                                                         const int* __restrict__ cells, int m,
                                                         __bf16* __restrict__ X,
                                                         float* __restrict__ target,
                                                         float* __restrict__ sigma) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, w = threadIdx.x >> 6;
  const int row = (blockIdx.x * 4 + w) * 16 + c;
  const bool ok = row < m;
  const int id = ok ? cells[row] : 0;
  const int x = id % geo.nx, y = (id / geo.nx) % geo.ny, z = id / (geo.nx * geo.ny);
  const NodeFeatures f = node_features(phi1, ux, uy, uz, geo, x, y, z, g);
  if (!ok) return;
  *reinterpret_cast<bf16x8*>(&X[(size_t)row * NF + 8 * g]) = f.x;
  if (g == 0) {
    target[row] = (phi_next[id] - f.centre) / f.sigma;
    sigma[row] = f.sigma;
  }
}

// Learned step, second half: out = Phi1 + sigma * net(features), limited to
// the range of the 27 values around the node.  A wave tile is 32 nodes of
// one x row (two MFMA tiles of 16).  Wave w of workgroup b takes the tiles
// 4b + w, 4b + w + 4G, ... (G workgroups); every workgroup loads the weights
// into LDS once, after which its waves run independently.
struct InferLds {
  WeightsLds W;
  __bf16 h1[4][32 * SH];
};

__global__ __launch_bounds__(kThreads) void k_learned_correct(const float* __restrict__ phi1,
                                                              const float* __restrict__ ux,
                                                              const float* __restrict__ uy,
                                                              const float* __restrict__ uz,
                                                              Geo geo,
                                                              const __bf16* __restrict__ wpack,
                                                              const float* __restrict__ wr,
                                                              float* __restrict__ out, bool fast) {
  extern __shared__ __align__(16) unsigned char smem[];
  InferLds& L = *reinterpret_cast<InferLds*>(smem);
  load_weights(L.W, nullptr, wpack, wr);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, w = threadIdx.x >> 6;
  const int nxb = (geo.nx + 31) / 32;
  const int tiles = nxb * geo.ny * geo.nz;
  constexpr int WPB = kThreads / 64;
  // byte offsets of this lane's neighbours from the node, computed once, and
  // which of them step across the low (m) or high (p) face of each axis
  const size_t ncells = (size_t)geo.nx * geo.ny * geo.nz;
  const unsigned plane = unsigned(geo.nx) * unsigned(geo.ny);
  const Rsrc rp = field_rsrc(phi1, ncells), rx = field_rsrc(ux, ncells);
  const Rsrc ry = field_rsrc(uy, ncells), rz = field_rsrc(uz, ncells);
  int noff[8];
  unsigned xm = 0, xp = 0, ym = 0, yp = 0, zm = 0, zp = 0;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int k = min(8 * g + v, 26);
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    noff[v] = 4 * (dz * int(plane) + dy * geo.nx + dx);
    xm |= unsigned(dx < 0) << v;
    xp |= unsigned(dx > 0) << v;
    ym |= unsigned(dy < 0) << v;
    yp |= unsigned(dy > 0) << v;
    zm |= unsigned(dz < 0) << v;
    zp |= unsigned(dz > 0) << v;
  }
  // a neighbour across a face is the node on the opposite face (periodic):
  // one axis length further along that axis
  const unsigned wx4 = 4u * unsigned(geo.nx), wy4 = 4u * plane, wz4 = 4u * unsigned(ncells);
  for (int t = blockIdx.x * WPB + w; t < tiles; t += gridDim.x * WPB) {
    const int tu = __builtin_amdgcn_readfirstlane(t);  // the same for the whole wave
    const int xb0 = (tu % nxb) * 32;
    const int row = tu / nxb;
    const int y = row % geo.ny, z = row / geo.ny;
    bf16x8 xb[2];
    float sig[2], cen[2], lo[2], hi[2];
    int xs[2];
    // wrap corrections of the tile's row (the same for every node of the row)
    const unsigned ysel = y == 0 ? ym : (y == geo.ny - 1 ? yp : 0u);
    const unsigned ydel = y == 0 ? wy4 : 0u - wy4;
    const unsigned zsel = z == 0 ? zm : (z == geo.nz - 1 ? zp : 0u);
    const unsigned zdel = z == 0 ? wz4 : 0u - wz4;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      xs[jt] = xb0 + 16 * jt + c;
      const int x = min(xs[jt], geo.nx - 1);  // lanes past the end repeat the last node
      NodeFeatures f;
      if (fast) {
        const unsigned ic4 = 4u * (unsigned(z) * plane + unsigned(y) * unsigned(geo.nx) + unsigned(x));
        const unsigned xsel = x == 0 ? xm : (x == geo.nx - 1 ? xp : 0u);
        const unsigned xdel = x == 0 ? wx4 : 0u - wx4;
        float val[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          unsigned o = ic4 + unsigned(noff[v]);
          o += (xsel >> v & 1u) ? xdel : 0u;
          o += (ysel >> v & 1u) ? ydel : 0u;
          o += (zsel >> v & 1u) ? zdel : 0u;
          val[v] = ld_at(rp, o);
        }
        f = features_from(val, ld_at(rp, ic4), g, ld_at(rx, ic4) * geo.lam[0],
                          ld_at(ry, ic4) * geo.lam[1], ld_at(rz, ic4) * geo.lam[2]);
      } else {
        f = node_features(phi1, ux, uy, uz, geo, x, y, z, g);
      }
      xb[jt] = f.x;
      sig[jt] = f.sigma;
      cen[jt] = f.centre;
      lo[jt] = f.lo;
      hi[jt] = f.hi;
    }
    floatx4 h2[4][2];
    float yv[2];
    forward_tile(L.W, xb, L.h1[w], h2, yv);
    if (g == 0) {
#pragma unroll
      for (int jt = 0; jt < 2; ++jt)
        if (xs[jt] < geo.nx)
          out[(size_t)z * geo.nx * geo.ny + (size_t)y * geo.nx + xs[jt]] =
              fminf(fmaxf(fmaf(sig[jt], yv[jt], cen[jt]), lo[jt]), hi[jt]);
    }
  }
}


// ---------------------------------------------------------------------------
// Learned step, second half, as a march along z (the default).  A workgroup
// of kLmRows waves owns a window of 64 consecutive x by kLmRows rows of y and
// marches along z through a chunk of planes.  Every plane of the CIR field
// is staged in LDS over the window plus one node on each side and the rows
// plus one on each side (a ring of 4 planes, so one barrier per plane); each
// lane then builds the features of one node from the 27 staged values
// around it.  The features reach the matrix-core operand layout by a
// transpose across the wave's 16-lane rows on the vector ALU, and the
// network runs on the wave's 64 nodes at once.
//
// The hidden units of the first layer are computed in a permuted row order
// (W1's columns and b1 are permuted when they are staged): matrix-core tile
// `it` row 4g + q of the first layer holds hidden unit
// 32 (it / 2) + 8 g + 4 (it % 2) + q, which is exactly the unit lane (g, c)
// supplies as operand element j = 4 (it % 2) + q of the second layer's
// K-block it / 2.  So the first layer's results feed the second layer from
// the lanes that hold them: no exchange through LDS.  Row permutations do
// not change how any one output is accumulated, so per node the FP32
// operations and their order are those of k_learned_correct: the same
// results bit for bit.
// ---------------------------------------------------------------------------
constexpr int kLmRows = 8, kLmX = 64, kLmW = kLmX + 2, kLmH = kLmRows + 2, kLmRing = 4;
constexpr int kLmThreads = 64 * kLmRows;
struct MarchLds {
  __bf16 w1t[NH * SF];  // permuted rows (see above)
  __bf16 w2t[NH * SH];
  float b1[NH];         // permuted like W1's rows
  float b2[NH], w3[NH], b3;
  float phi[kLmRing][kLmH][kLmW];
};
static_assert(offsetof(MarchLds, b1) % 16 == 0 && offsetof(MarchLds, b2) % 16 == 0,
              "bias rows must be 16-byte aligned");

// Hidden unit computed by permuted first-layer row r.
__device__ __forceinline__ int lm_unit(int r) {
  const int it = r / 16, g = (r % 16) / 4, q = r % 4;
  return 32 * (it / 2) + 8 * g + 4 * (it % 2) + q;
}

// Buffer access at a per-lane byte offset voff from the row that starts soff
// bytes into the field (soff the same for the whole wave): the descriptor is
// rebased on the row (two scalar adds) and has the largest size a descriptor
// holds, so voff alone is range-checked.
__device__ __forceinline__ Rsrc row_rsrc(const float* field, unsigned soff) {
  const size_t off = unsigned(__builtin_amdgcn_readfirstlane(int(soff)));
  const char* b = reinterpret_cast<const char*>(field) + off;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), short(0), int(0xFFFFFFFFu), 0x00020000);
}
__device__ __forceinline__ float ld_row(const float* field, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(field, soff), voff, 0, 0));
}
__device__ __forceinline__ void st_row(float* field, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), row_rsrc(field, soff), voff,
                                        0, 0);
}

// wrap any coordinate into [0, n)
__device__ __forceinline__ int wrapk(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

__global__ __launch_bounds__(kLmThreads, 4) void k_learned_march(const float* __restrict__ phi1,
                                                              const float* __restrict__ ux,
                                                              const float* __restrict__ uy,
                                                              const float* __restrict__ uz, Geo geo,
                                                              const __bf16* __restrict__ wpack,
                                                              const float* __restrict__ wr,
                                                              float* __restrict__ out, int chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  MarchLds& L = *reinterpret_cast<MarchLds*>(smem);
  for (int i = threadIdx.x; i < NH * NF; i += kLmThreads) {
    const int r = i / NF, k = i % NF;
    L.w1t[r * SF + k] = wpack[lm_unit(r) * NF + k];
  }
  for (int i = threadIdx.x; i < NH * NH; i += kLmThreads)
    L.w2t[(i / NH) * SH + i % NH] = wpack[NH * NF + i];
  for (int i = threadIdx.x; i < NH; i += kLmThreads) {
    L.b1[i] = wr[B1_OFF + lm_unit(i)];
    L.b2[i] = wr[B2_OFF + i];
    L.w3[i] = wr[W3_OFF + i];
  }
  if (threadIdx.x == 0) L.b3 = wr[B3_OFF];
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15, w = threadIdx.x >> 6;
  const int nx = geo.nx, ny = geo.ny, nz = geo.nz;
  const int nwx = (nx + kLmX - 1) / kLmX, nry = (ny + kLmRows - 1) / kLmRows;
  const int b = blockIdx.x;
  const int wx = b % nwx, ry = (b / nwx) % nry, ch = b / (nwx * nry);
  const int x0 = wx * kLmX, y0 = ry * kLmRows, z0 = ch * chunk, z1 = min(z0 + chunk, nz);
  // Global accesses: a byte offset per lane (its x) and a row offset that is
  // the same for the whole wave (scalar registers); fields of at most 2^30
  // cells keep both below 2^32.
  const unsigned rowb = 4u * unsigned(nx);
  // this lane's x (wrapped, so the lanes past a short row hold the nodes
  // that follow it periodically) and the two halo nodes (lanes 0 and 1)
  const unsigned vxl = 4u * unsigned(wrapk(x0 + lane, nx));
  // the halo nodes' offsets: two scalars, chosen per lane where used (a
  // per-lane register held across the march does not fit)
  const unsigned hxm = 4u * unsigned(__builtin_amdgcn_readfirstlane(wrapk(x0 - 1, nx)));
  const unsigned hxp = 4u * unsigned(__builtin_amdgcn_readfirstlane(wrapk(x0 + kLmX, nx)));
  // staged rows: wave w loads row w of y0 - 1 .. y0 + kLmRows, waves 0 and 1
  // also rows kLmRows and kLmRows + 1
  int srow[2];
  srow[0] = __builtin_amdgcn_readfirstlane(wrapk(y0 - 1 + w, ny));
  srow[1] = __builtin_amdgcn_readfirstlane(wrapk(y0 - 1 + w + kLmRows, ny));
  const int nsr = w + kLmRows < kLmH ? 2 : 1;
  const int y = y0 + w;  // this wave's output row
  const bool lane_ok = y < ny && x0 + lane < nx;
  const int yc = __builtin_amdgcn_readfirstlane(min(y, ny - 1));
  float pre[2], preh[2];
  auto fetch = [&](int zp) {  // the staged rows of plane zp (wrapped)
    const unsigned pz = unsigned(__builtin_amdgcn_readfirstlane(wrapk(zp, nz))) * unsigned(ny);
    // Every load is unconditional (a load under a condition would make the
    // wave wait for it at once): the waves that stage one row load a second,
    // valid, row that goes unused, and lanes past 1 load their own node again
    // as the unused halo value.
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const unsigned row = (pz + unsigned(srow[r])) * rowb;
      pre[r] = ld_row(phi1, vxl, row);
      int ln = lane;
      asm volatile("" : "+v"(ln));  // recomputes the choice here, every plane
      preh[r] = ld_row(phi1, ln == 0 ? hxm : ln == 1 ? hxp : vxl, row);
    }
  };
  auto stage = [&](int slot) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (r < nsr) {
        float* dst = L.phi[slot][w + kLmRows * r];
        dst[lane + 1] = pre[r];
        if (lane == 0) dst[0] = preh[r];
        if (lane == 1) dst[kLmW - 1] = preh[r];
      }
    }
  };
  // planes z0 - 1 and z0 in slots 0 and 1; plane z0 + 1 in flight
  fetch(z0 - 1);
  stage(0);
  fetch(z0);
  stage(1);
  fetch(z0 + 1);
  __syncthreads();  // the weights
  float w3r[4][4];  // w3 of the second layer's outputs this lane holds
#pragma unroll
  for (int it = 0; it < 4; ++it)
#pragma unroll
    for (int q = 0; q < 4; ++q) w3r[it][q] = L.w3[16 * it + 4 * g + q];
  const float b3 = L.b3;
  for (int z = z0; z < z1; ++z) {
    const int t = z - z0;  // plane z sits in slot (t + 1) % 4
    stage((t + 2) % kLmRing);  // plane z + 1
    // node velocity of this lane (only its Courant numbers are features),
    // loaded before the next plane's rows: loads complete in order, so the
    // wait for these leaves that fetch in flight
    const unsigned rowz = (unsigned(z) * unsigned(ny) + unsigned(yc)) * rowb;
    const float ucx = ld_row(ux, vxl, rowz), ucy = ld_row(uy, vxl, rowz), ucz = ld_row(uz, vxl, rowz);
    fetch(z + 2);  // in flight while this plane's nodes run
    const float cx = ucx * geo.lam[0], cy = ucy * geo.lam[1], cz = ucz * geo.lam[2];
    __syncthreads();
    // the 27 values around this lane's node: slots of planes z-1, z, z+1,
    // staged rows w .. w + 2, x positions lane .. lane + 2
    float val[27];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      const float* sp = &L.phi[(t + dz) & (kLmRing - 1)][w][lane];
#pragma unroll
      for (int k = 0; k < 9; ++k) val[9 * dz + k] = sp[(k / 3) * kLmW + k % 3];
    }
    const float centre = val[13];
    float lo = centre, hi = centre, ssg[4], d[27];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ssg[q] = 0.f;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int k = 8 * q + v;
        if (k < 27) {
          lo = fminf(lo, val[k]);
          hi = fmaxf(hi, val[k]);
          d[k] = val[k] - centre;
          ssg[q] = fmaf(d[k], d[k], ssg[q]);
        }
      }
    }
    const float ss = (ssg[0] + ssg[1]) + (ssg[2] + ssg[3]);
    const float sigma = sqrtf(ss / 27.f + 1e-30f);
    const float inv = 1.f / sigma;
    float fv[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      fv[k] = 0.f;
      if (k < 27) fv[k] = d[k] * inv;
      else if (k == 27) fv[k] = cx;
      else if (k == 28) fv[k] = cy;
      else if (k == 29) fv[k] = cz;
    }
    // chunk j: features 8j..8j+7 of this lane's node (node 16 g + c)
    uintx4 ch[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int h = 0; h < 4; ++h) ch[j][h] = cvt_pk_bf16(fv[8 * j + 2 * h], fv[8 * j + 2 * h + 1]);
    // The matrix-core operand of node tile jt on lane (g, c) is chunk g of
    // node 16 jt + c, held by lane (jt, c): a 4 x 4 transpose of chunks
    // across the four 16-lane rows, done with gfx950's row swaps between
    // register pairs (rows r and r ^ 1, then rows r and r ^ 2) on the vector
    // ALU instead of a round trip through LDS.
    uintx4 xt[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const uintx2 p01 = __builtin_amdgcn_permlane16_swap(ch[0][h], ch[1][h], false, false);
      const uintx2 p23 = __builtin_amdgcn_permlane16_swap(ch[2][h], ch[3][h], false, false);
      const uintx2 q02 = __builtin_amdgcn_permlane32_swap(p01[0], p23[0], false, false);
      const uintx2 q13 = __builtin_amdgcn_permlane32_swap(p01[1], p23[1], false, false);
      unsigned r[4] = {q02[0], q13[0], q02[1], q13[1]};
      asm("" : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]));  // see the sum below
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) xt[jt][h] = r[jt];
    }
    bf16x8 xb[4];  // node tile jt: features 8g..8g+7 of node 16 jt + c
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) xb[jt] = __builtin_bit_cast(bf16x8, xt[jt]);
    // layer 1 (permuted rows), BF16, ReLU: the second layer's operands in place
    uintx4 h1[4][2];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const bf16x8 a = ld8(&L.w1t[(16 * it + c) * SF + 8 * g]);
      const floatx4 bias = *reinterpret_cast<const floatx4*>(&L.b1[16 * it + 4 * g]);
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) {
        const floatx4 acc = mfma(a, xb[jt], bias);
        h1[jt][it / 2][2 * (it % 2)] = relu_pk(cvt_pk_bf16(acc[0], acc[1]));
        h1[jt][it / 2][2 * (it % 2) + 1] = relu_pk(cvt_pk_bf16(acc[2], acc[3]));
      }
    }
    // layer 2, ReLU, and the output layer's dot product
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const bf16x8 a0 = ld8(&L.w2t[(16 * it + c) * SH + 8 * g]);
      const bf16x8 a1 = ld8(&L.w2t[(16 * it + c) * SH + 32 + 8 * g]);
      const floatx4 bias = *reinterpret_cast<const floatx4*>(&L.b2[16 * it + 4 * g]);
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) {
        floatx4 acc = mfma(a0, __builtin_bit_cast(bf16x8, h1[jt][0]), bias);
        acc = mfma(a1, __builtin_bit_cast(bf16x8, h1[jt][1]), acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) s[jt] = fmaf(relu_bits(acc[q]), w3r[it][q], s[jt]);
      }
    }
    // y of node `lane` (16 g + c): the four partial sums of that node are
    // s[g] on the lanes (j, c), j = 0..3; the same row transpose brings them
    // to this lane as ps[j], added in the order of sum4g ((0+1) + (2+3))
    float ps[4];
    {
      const uintx2 p01 = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, s[0]),
                                                          __builtin_bit_cast(unsigned, s[1]), false, false);
      const uintx2 p23 = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, s[2]),
                                                          __builtin_bit_cast(unsigned, s[3]), false, false);
      const uintx2 q02 = __builtin_amdgcn_permlane32_swap(p01[0], p23[0], false, false);
      const uintx2 q13 = __builtin_amdgcn_permlane32_swap(p01[1], p23[1], false, false);
      unsigned r[4] = {q02[0], q13[0], q02[1], q13[1]};
      // the compiler takes the two results of a row swap to be
      // interchangeable in a sum and folds (a + b) + (c + d) into 2 (a + b):
      // empty asm statements keep the four values apart
      asm("" : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]));
#pragma unroll
      for (int j = 0; j < 4; ++j) ps[j] = __builtin_bit_cast(float, r[j]);
    }
    const float yn = ((ps[0] + ps[1]) + (ps[2] + ps[3])) + b3;
    if (lane_ok) st_row(out, vxl, rowz, fminf(fmaxf(fmaf(sigma, yn, centre), lo), hi));
  }
}
}  // namespace

size_t mlp_train_lds() { return sizeof(TrainLds); }

hipError_t launch_mlp(bool train, const void* X, const float* target, int m, float inv_m2,
                      const void* wpack, const float* wr, float* yout, float* gpart,
                      float* lpart, int* nblk_out, hipStream_t st) {
  const int tiles = (m + 31) / 32;
  if (!train) {
    // enough blocks to fill the chip, each wave running tiles_per_wave tiles
    const int tpw = max(1, (tiles + 4 * kMlpMaxBlocks - 1) / (4 * kMlpMaxBlocks));
    const int nblk = max(1, (tiles + 4 * tpw - 1) / (4 * tpw));
    if (nblk_out) *nblk_out = nblk;
    hipLaunchKernelGGL(k_mlp_eval, dim3(nblk), dim3(kThreads), 0, st, static_cast<const __bf16*>(X), m,
                       tpw, static_cast<const __bf16*>(wpack), wr, yout);
    return hipGetLastError();
  }
  // about one block per compute unit (one fits), at most the partials' room
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    cus = min(cus, kMlpMaxBlocks);
  }
  const int tpw = max(1, (tiles + kTrWaves * cus - 1) / (kTrWaves * cus));
  const int nblk = max(1, (tiles + kTrWaves * tpw - 1) / (kTrWaves * tpw));
  const int bytes = int(sizeof(TrainLds));
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_train),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (attr != hipSuccess) return attr;
  if (nblk_out) *nblk_out = nblk;
  hipLaunchKernelGGL(k_mlp_train, dim3(nblk), dim3(64 * kTrWaves), bytes, st,
                     static_cast<const __bf16*>(X), target, m, inv_m2, tpw,
                     static_cast<const __bf16*>(wpack), wr, gpart, lpart);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* gpart, const float* lpart, int nblk, float* grad,
                              double* loss_sum, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_reduce<false>, dim3((kMlpParams + kRedParams - 1) / kRedParams),
                     dim3(kThreads), 0, st, gpart, lpart, nblk, grad, loss_sum, AdamArgs{});
  return hipGetLastError();
}

hipError_t launch_grad_adam(const float* gpart, const float* lpart, int nblk, float* grad,
                            double* loss_sum, float* master, float* m, float* v, float lr,
                            float beta1, float beta2, float eps, float bc1, float bc2, float* wr,
                            void* wpack, hipStream_t st) {
  const AdamArgs ad{master, m, v, lr, beta1, beta2, eps, bc1, bc2, wr, static_cast<__bf16*>(wpack)};
  hipLaunchKernelGGL(k_grad_reduce<true>, dim3((kMlpParams + kRedParams - 1) / kRedParams),
                     dim3(kThreads), 0, st, gpart, lpart, nblk, grad, loss_sum, ad);
  return hipGetLastError();
}

hipError_t launch_pack(const float* master, float* wr, void* wpack, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3((kMlpParams + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     master, wr, static_cast<__bf16*>(wpack));
  return hipGetLastError();
}

hipError_t launch_make_pairs(const Geo& g, const float* phi1, const float* phi_next, const float* u,
                             const int* cells, int m, void* X, float* target, float* sigma,
                             hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  const int nblk = (m + 63) / 64;
  hipLaunchKernelGGL(k_make_pairs, dim3(nblk), dim3(kThreads), 0, st, phi1, phi_next, u, u + n,
                     u + 2 * n, g, cells, m, static_cast<__bf16*>(X), target, sigma);
  return hipGetLastError();
}

hipError_t launch_learned_march(const Geo& g, const float* phi1, const float* u, const void* wpack,
                                const float* wr, float* out, hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  // row offsets are 32-bit: fields of 2^30 cells take the gather
  if (n >= (size_t(1) << 30)) return launch_learned_correct(g, phi1, u, wpack, wr, out, st);
  const int bytes = int(sizeof(MarchLds));
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(k_learned_march),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (attr != hipSuccess) return attr;
  const long long cols = (long long)((g.nx + kLmX - 1) / kLmX) * ((g.ny + kLmRows - 1) / kLmRows);
  // march chunks of 32 planes, or shorter if that leaves under 2048 workgroups
  int chunk = 32;
  while (chunk > 8 && cols * ((g.nz + chunk - 1) / chunk) < 2048) chunk /= 2;
  const long long blocks = cols * ((g.nz + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_learned_march, dim3(unsigned(blocks)), dim3(kLmThreads), bytes, st, phi1, u,
                     u + n, u + 2 * n, g, static_cast<const __bf16*>(wpack), wr, out, chunk);
  return hipGetLastError();
}

hipError_t launch_learned_correct(const Geo& g, const float* phi1, const float* u, const void* wpack,
                                  const float* wr, float* out, hipStream_t st) {
  const size_t n = (size_t)g.ncells;
  const int bytes = int(sizeof(InferLds));
  const long long wave_tiles = (long long)((g.nx + 31) / 32) * g.ny * g.nz;
  const int blocks = int(std::min<long long>((wave_tiles + 3) / 4, kLearnedBlocks));
  hipLaunchKernelGGL(k_learned_correct, dim3(blocks), dim3(kThreads), bytes, st, phi1, u, u + n, u + 2 * n,
                     g, static_cast<const __bf16*>(wpack), wr, out, n < (size_t(1) << 30));
  return hipGetLastError();
}

}  // namespace sla
