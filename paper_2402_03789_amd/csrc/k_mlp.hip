// Fused radial MLP on the matrix cores: the BF16 form with bfloat16 operands and storage,
// the FP32 form with float32 storage and its two P-wide contractions in three-part
// bfloat16 arithmetic (float32-level results; the split kernels below).
//
// Per undirected edge pair (paper section 5.1, "learnable radial functions"
// of the 8 Bessel features; the weights depend only on the distance, so an
// edge and its reverse share them):
//   a1 = rho Wa,  z1 = phi(a1),  a2 = z1 Wb,  z2 = phi(a2),  w = z2 Wc
// with phi(z) = c z sigmoid(z) and no biases.  The adjoint maps
// dE/dw = dw[2p] + dw[2p+1] (both directions of pair p, stored in adjacent rows) back to
// dE/drho:
//   dz2 = dw Wc^T,  da2 = dz2 phi'(a2),  dz1 = da2 Wb^T,  da1 = dz1 phi'(a1),
//   drho = da1 Wa^T   (hidden activations recomputed; drho lands on edge e1).
//
// One 256-thread block = 64 pairs; each of the 4 waves owns 16 pairs and
// computes 16 x 64 output panels as four 16 x 16 MFMA tiles.  Hidden
// activations stay on the CU (registers and a per-wave LDS panel that turns
// the accumulator layout into the operand layout); weight panels are staged
// in LDS once per block and shared by the four waves.  The output layer is
// computed transposed (w^T = Wc^T z2^T), so a lane's accumulators hold
// consecutive weights of one pair; they leave through the wave's LDS panel so
// that each 16-byte store instruction writes whole row segments.  The adjoint
// reads dE/dw row-coalesced and turns it into the operand layout through the
// wave's LDS panel.
//
// MFMA layouts (lane l, 16 x 16 tiles):
//   f32 16x16x4  : a = A[l%16][4s + l/16],     b = B[4s + l/16][l%16]
//   bf16 16x16x32: a = A[l%16][32s + 8(l/16) + 0..7], b = B[32s + 8(l/16) + 0..7][l%16]
//   result       : acc[r] = C[4(l/16) + r][l%16]
// LDS strides: operand panels 68 floats, k-major weight panels 80 floats, chosen so
// that the 64 lanes of a fragment read hit distinct banks.
#include "kernels.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace sn {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <class F, int... I>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int EB = 64;   // pairs per block
constexpr int HID = 64;  // hidden width
constexpr int NBAS = 8;  // radial features
constexpr int ZP = 68;   // operand panel stride (floats)
constexpr int WP = 80;   // k-major weight panel stride (floats)
constexpr int BP = 72;   // n-major bf16 panel stride (16-byte aligned rows)

__device__ inline float phi(float z, float c) { return c * z / (1.f + __expf(-z)); }
__device__ inline float dphi(float z, float c) {
  float s = 1.f / (1.f + __expf(-z));
  return c * (s + z * s * (1.f - s));
}

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline void zero4(floatx4 a[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) a[t] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// acc += Z(16 x 64 operand panel) * W, W k-major [k][n] (stride WP)
__device__ inline void panel_kn(const float* Z, const float* W, floatx4 acc[4], int lane) {
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int s = 0; s < HID / 4; ++s) {
    const float a = Z[r * ZP + 4 * s + q];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma4(a, W[(4 * s + q) * WP + t * 16 + r], acc[t]);
  }
}

// acc += Z * W^T with W k-major [n][k] as stored for the forward product (B[k][n] = W[n][k])
__device__ inline void panel_kn_T(const float* Z, const float* W, floatx4 acc[4], int lane) {
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int s = 0; s < HID / 4; ++s) {
    const float a = Z[r * ZP + 4 * s + q];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma4(a, W[(t * 16 + r) * WP + 4 * s + q], acc[t]);
  }
}

// bfloat16 form of the hidden 64 x 64 products: acc += Z * B with Z the float operand
// panel (rounded to bfloat16 as it is read) and B^T stored as bfloat16 rows [n][k]
// (stride BP), two 16x16x32 steps per tile
__device__ inline void panel_bf16(const float* Z, const __bf16* Bt, floatx4 acc[4], int lane) {
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int s = 0; s < HID / 32; ++s) {
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = __float2bfloat16(Z[r * ZP + 32 * s + 8 * q + e]);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = mfma32(a, *reinterpret_cast<const bf16x8*>(&Bt[(t * 16 + r) * BP + 32 * s + 8 * q]),
                      acc[t]);
  }
}
// Wb staged as bfloat16 B^T panels: for z1 Wb (bt[n][k] = Wb[k][n]) and, when wanted, for
// da2 Wb^T (bn[n][k] = Wb[n][k])
__device__ inline void stage_wb_bf16(const float* __restrict__ Wb, __bf16* bt, __bf16* bn) {
  for (int i = threadIdx.x; i < HID * HID; i += 256) {
    const int k = i / HID, n = i % HID;  // Wb[k][n]
    const __bf16 v = __float2bfloat16(Wb[i]);
    bt[n * BP + k] = v;
    if (bn) bn[k * BP + n] = v;
  }
}

// accumulator tiles (16 x 64) -> operand panel, applying f(v, tile, row)
template <class F>
__device__ inline void acc_to_panel(const floatx4 acc[4], float* Z, int lane, F&& f) {
  const int c = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) Z[(rq + rr) * ZP + t * 16 + c] = f(acc[t][rr], t, rr);
}

// a1 (accumulator layout) = rho(16 x 8) Wa(8 x 64); rho panel stride NBAS + 1
__device__ inline void first_layer(const float* sRho, const float* sWa, floatx4 acc[4], int lane) {
  const int r = lane & 15, q = lane >> 4;
  zero4(acc);
#pragma unroll
  for (int s = 0; s < NBAS / 4; ++s) {
    const float a = sRho[r * (NBAS + 1) + 4 * s + q];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma4(a, sWa[(4 * s + q) * HID + t * 16 + r], acc[t]);
  }
}

__device__ inline void stage_common(int64_t np, int64_t p0, const int* __restrict__ pe1,
                                    const float* __restrict__ rho, const float* __restrict__ Wa,
                                    const float* __restrict__ Wb, float* sWa, float* sWb,
                                    float* sRho) {
  const int tid = threadIdx.x;
  for (int i = tid; i < NBAS * HID; i += 256) sWa[i] = Wa[i];
  if (sWb)
    for (int i = tid; i < HID * HID; i += 256) sWb[(i / HID) * WP + i % HID] = Wb[i];
  for (int i = tid; i < EB * NBAS; i += 256) {
    const int64_t p = p0 + i / NBAS;
    sRho[(i / NBAS) * (NBAS + 1) + i % NBAS] = p < np ? rho[(int64_t)pe1[p] * NBAS + i % NBAS] : 0.f;
  }
}

// Output-layer weights Wc [64 x P] arrive rearranged into 64-column panels, each a
// contiguous 64 x 64 block of bfloat16 (zero past column P): [panel][j][c] (hidden row j,
// column c) for the adjoint, transposed per panel, [panel][c][j], for the forward (the
// FP32 form's three-part copies are described with its kernels).  A panel is staged into
// LDS through registers: each of the 256 threads loads 16 bytes per step (two steps) while
// the current panel is being multiplied, and stores them as 16-byte segments of the LDS
// panel's rows (stride BP).  Loads past the last panel read the last one again (valid
// memory; the copy is never used).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct PanelRegs {
  u32x4 v[2];
};
constexpr int kPanel = HID * HID;  // elements per panel

__device__ inline void fetch_panel(const bf16_t* __restrict__ pan, int panel, int npan, int tid,
                                   PanelRegs& r) {
  const bf16_t* src = pan + (int64_t)min(panel, npan - 1) * kPanel;
#pragma unroll
  for (int j = 0; j < 2; ++j) r.v[j] = *reinterpret_cast<const u32x4*>(src + (tid + 256 * j) * 8);
}
__device__ inline void store_panel(const PanelRegs& r, int tid, void* lds) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int i = (tid + 256 * j) * 8;
    *reinterpret_cast<u32x4*>(reinterpret_cast<__bf16*>(lds) + (i / HID) * BP + i % HID) = r.v[j];
  }
}

// ------------------------------------------------------------------ forward
template <bool BF16>
using WStore = typename std::conditional<BF16, bf16_t, float>::type;

// BF16 form (the FP32 form's output layer is the split kernel below)
__global__ __launch_bounds__(256) void k_mlp_fused_fwd(int64_t np, const int* __restrict__ pe1,
                                                        const float* __restrict__ rho,
                                                        const float* __restrict__ Wa,
                                                        const float* __restrict__ Wb,
                                                        const bf16_t* __restrict__ Wcp, int P,
                                                        float c, bf16_t* __restrict__ w) {
  __shared__ float sWa[NBAS * HID];
  __shared__ float sRho[EB * (NBAS + 1)];
  __shared__ float sZ[4][16 * ZP];
  // two bfloat16 Wc panel stages of row stride BP; the second one holds Wb (bfloat16 B^T
  // rows) for the hidden layers first.  About 40 KB of LDS: four blocks per CU.
  __shared__ __attribute__((aligned(16))) float sW[2][HID * BP / 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  // output panels of this block: all of them, or (few pairs) one of gridDim.y panel groups;
  // each group recomputes the pairs' hidden layers, which are cheap next to the panels
  const int npan = (P + HID - 1) / HID;
  const int ppg = (npan + gridDim.y - 1) / gridDim.y;
  const int pan0 = blockIdx.y * ppg, pan1 = min(npan, pan0 + ppg);
  if (pan0 >= pan1) return;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, nullptr, sRho);
  __bf16* sWbT = reinterpret_cast<__bf16*>(sW[1]);
  stage_wb_bf16(Wb, sWbT, nullptr);
  PanelRegs pr;
  fetch_panel(Wcp, pan0, npan, tid, pr);
  __syncthreads();
  float* Z = sZ[wave];
  floatx4 acc[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, acc, lane);
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  store_panel(pr, tid, sW[0]);
  __syncthreads();
  zero4(acc);
  panel_bf16(Z, sWbT, acc, lane);
  __syncthreads();
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  __syncthreads();
  // z2 operand fragments, kept in registers for every output panel
  const int r = lane & 15, q = lane >> 4;
  bf16x8 zh[HID / 32];
#pragma unroll
  for (int s = 0; s < HID / 32; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) zh[s][e] = __float2bfloat16(Z[r * ZP + 32 * s + 8 * q + e]);
  // Wc panels in flight: a ring of RING register sets, RING - 1 panels ahead of the one
  // being multiplied (a panel's eight MFMAs per wave take far less than the L2 round trip
  // of the next panel's loads).  Panel pan0 + k travels in ring slot k % RING; the loop is
  // unrolled by RING so the slots are fixed registers.
  constexpr int RING = 3;
  PanelRegs ring[RING];
  const int count = pan1 - pan0;
  static_for<RING - 1>([&](auto J) {
    constexpr int k = decltype(J)::value + 1;
    fetch_panel(Wcp, pan0 + k, npan, tid, ring[k % RING]);
  });
  int buf = 0;
  auto step = [&](int jj, auto SLOT) {
    constexpr int sc = decltype(SLOT)::value, sn = (sc + 1) % RING;
    // slot sc held panel jj, staged into LDS by the previous step: reuse it for panel
    // jj + RING (loads past the last panel read the last one again and are never used)
    fetch_panel(Wcp, pan0 + jj + RING, npan, tid, ring[sc]);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
    const __bf16* sh = reinterpret_cast<const __bf16*>(sW[buf]);
    const int n0 = (pan0 + jj) * HID;
    // the transposed product w^T = Wc^T z2^T: lane (r, q) receives weights of pair r only;
    // row i of tile t is panel column 16 (i / 4) + 4 t + i % 4, so acc[0..3][0..3] =
    // w[pair r][n0 + 16 q + 0..15]
    zero4(acc);
    if (jj < count) {
      const int ca = 16 * (r >> 2) + (r & 3);
#pragma unroll
      for (int s = 0; s < HID / 32; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sh[(ca + 4 * t) * BP + 32 * s + 8 * q]);
          acc[t] = mfma32(a, zh[s], acc[t]);
        }
    }
    // staged unconditionally (a panel past the last is never read): a conditional store
    // would let the compiler sink the panel loads into the branch, after the MFMAs
    store_panel(ring[sn], tid, sW[buf ^ 1]);
    // out through the wave's LDS tile (free once z2 is in registers): a 16-byte store then
    // writes eight whole 128-byte row segments instead of pieces of sixteen rows.  LDS
    // operations of one wave complete in order; the empty asm statements keep the compiler
    // from moving the tile's reads across its writes.
    if (jj < count) {
      __bf16* Zb = reinterpret_cast<__bf16*>(Z);  // rows of 2 ZP bfloat16 values
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        u32x4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = 2 * h + (e >> 1), rr = 2 * (e & 1);
          v[e] = (uint32_t)sstore<bf16_t>(acc[t][rr]).u |
                 ((uint32_t)sstore<bf16_t>(acc[t][rr + 1]).u << 16);
        }
        *reinterpret_cast<u32x4*>(Zb + r * 2 * ZP + 16 * q + 8 * h) = v;
      }
      __asm__ volatile("" ::: "memory");
      const int cb = 8 * (lane & 7);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int rr = 8 * k + (lane >> 3);
        const u32x4 v = *reinterpret_cast<const u32x4*>(Zb + rr * 2 * ZP + cb);
        const int64_t p = p0 + wave * 16 + rr;
        if (p < np && n0 + cb < P) *reinterpret_cast<u32x4*>(&w[p * P + n0 + cb]) = v;  // P % 8 == 0
      }
      __asm__ volatile("" ::: "memory");
    }
    __syncthreads();
    buf ^= 1;
  };
  for (int j = 0; j < count; j += RING) {
    static_for<RING>([&](auto J) { step(j + decltype(J)::value, J); });
  }
}

// ------------------------------------------------------------------ forward, split form
// The FP32 form's output layer in three-part bfloat16 arithmetic: every float32 operand x
// is written as x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1)
// (each difference exact in float32), which carries x's 24-bit significand.  The product
// a b is the sum of the six part products a_i b_j with i + j <= 2 (the dropped ones are
// below 2^-24 relative), each exact in the float32 accumulation of the bfloat16 matrix
// cores: float32-level results in 6 bfloat16 MFMAs per 32-wide k step instead of 8 float32
// ones at an eighth of the rate.  The hidden layers (6 % of the work) stay float32.
// Wc3 holds per panel the three parts, each transposed [c][j] (a 64 x 64 bfloat16 block).
constexpr int kPanel3 = 3 * HID * HID;  // elements per split panel
struct Panel3Regs {
  u32x4 v[6];
};
__device__ inline void fetch_panel3(const bf16_t* __restrict__ pan, int panel, int npan, int tid,
                                    Panel3Regs& r) {
  const bf16_t* src = pan + (int64_t)min(panel, npan - 1) * kPanel3;
#pragma unroll
  for (int j = 0; j < 6; ++j) r.v[j] = *reinterpret_cast<const u32x4*>(src + (tid + 256 * j) * 8);
}
// parts at lds + part * HID * BP, rows of stride BP
__device__ inline void store_panel3(const Panel3Regs& r, int tid, __bf16* lds) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int i = (tid + 256 * j) * 8, part = i / kPanel, ii = i % kPanel;
    *reinterpret_cast<u32x4*>(lds + part * HID * BP + (ii / HID) * BP + ii % HID) = r.v[j];
  }
}
__device__ inline void split3(float v, __bf16& h0, __bf16& h1, __bf16& h2) {
  h0 = __float2bfloat16(v);
  const float r1 = v - (float)h0;
  h1 = __float2bfloat16(r1);
  h2 = __float2bfloat16(r1 - (float)h1);
}

// One LDS stage for the split panels (two barriers per panel): the hidden layers' Wb, Wa
// and rho live in the stage until the first panel replaces them, so a block takes 44 KB
// and three blocks share a CU.  Outputs leave through the wave's LDS tile, so each store
// writes four whole 256-byte row segments instead of sixteen rows' scattered pieces.
__global__ __launch_bounds__(256) void k_mlp_fused_fwd_split(int64_t np, const int* __restrict__ pe1,
                                                              const float* __restrict__ rho,
                                                              const float* __restrict__ Wa,
                                                              const float* __restrict__ Wb,
                                                              const bf16_t* __restrict__ Wc3, int P,
                                                              float c, float* __restrict__ w) {
  constexpr int kStage = 3 * HID * BP;  // bfloat16 elements of a split-panel stage
  __shared__ float sZ[4][16 * ZP];
  __shared__ __attribute__((aligned(16))) __bf16 sS[kStage];
  static_assert(sizeof(float) * (HID * WP + NBAS * HID + EB * (NBAS + 1)) <= sizeof(__bf16) * kStage,
                "the hidden layers' operands fit the stage");
  float* sWb = reinterpret_cast<float*>(sS);
  float* sWa = sWb + HID * WP;
  float* sRho = sWa + NBAS * HID;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  const int npan = (P + HID - 1) / HID;
  const int ppg = (npan + gridDim.y - 1) / gridDim.y;
  const int pan0 = blockIdx.y * ppg, pan1 = min(npan, pan0 + ppg);
  if (pan0 >= pan1) return;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, sWb, sRho);
  Panel3Regs pr;
  fetch_panel3(Wc3, pan0, npan, tid, pr);
  __syncthreads();
  float* Z = sZ[wave];
  floatx4 acc[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, acc, lane);
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  __syncthreads();
  zero4(acc);
  panel_kn(Z, sWb, acc, lane);
  __syncthreads();  // every wave is past Wb, Wa and rho: the stage takes the first panel
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  store_panel3(pr, tid, sS);
  __syncthreads();
  // z2 of pair r in three parts: eight consecutive k per lane and 32-wide step
  const int r = lane & 15, q = lane >> 4;
  bf16x8 z0[HID / 32], z1[HID / 32], z2[HID / 32];
#pragma unroll
  for (int st = 0; st < HID / 32; ++st)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 h0, h1, h2;
      split3(Z[r * ZP + 32 * st + 8 * q + e], h0, h1, h2);
      z0[st][e] = h0;
      z1[st][e] = h1;
      z2[st][e] = h2;
    }
  // w^T = Wc^T z2^T with the bfloat16 form's row order: row i of tile t is panel column
  // 16 (i / 4) + 4 t + i % 4, so acc[t] = w[pair r][n0 + 16 q + 4 t + 0..3]
  const int ca = 16 * (r >> 2) + (r & 3);
  // store layout: lane l writes columns 4 (l % 16) .. + 3 of the wave's rows l / 16 + 4 k
  const int cc = 4 * (lane & 15);
  for (int n0 = pan0 * HID; n0 < min(P, pan1 * HID); n0 += HID) {
    fetch_panel3(Wc3, n0 / HID + 1, npan, tid, pr);  // in flight during the MFMAs
    __builtin_amdgcn_sched_barrier(0);
    zero4(acc);
#pragma unroll
    for (int st = 0; st < HID / 32; ++st)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int off = (ca + 4 * t) * BP + 32 * st + 8 * q;
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(sS + off);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(sS + HID * BP + off);
        const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(sS + 2 * HID * BP + off);
        acc[t] = mfma32(a2, z0[st], acc[t]);  // smaller part products first
        acc[t] = mfma32(a1, z1[st], acc[t]);
        acc[t] = mfma32(a0, z2[st], acc[t]);
        acc[t] = mfma32(a1, z0[st], acc[t]);
        acc[t] = mfma32(a0, z1[st], acc[t]);
        acc[t] = mfma32(a0, z0[st], acc[t]);
      }
    // the wave's tile is its own: LDS operations of one wave complete in order, and the
    // empty asm statements keep the compiler from moving the tile's reads across its writes
#pragma unroll
    for (int t = 0; t < 4; ++t) *reinterpret_cast<floatx4*>(&Z[r * ZP + 16 * q + 4 * t]) = acc[t];
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rr = 4 * k + (lane >> 4);
      const floatx4 v = *reinterpret_cast<const floatx4*>(&Z[rr * ZP + cc]);
      const int64_t p = p0 + wave * 16 + rr;
      if (p < np && n0 + cc < P) *reinterpret_cast<floatx4*>(&w[p * P + n0 + cc]) = v;  // P % 4 == 0
    }
    __asm__ volatile("" ::: "memory");
    __syncthreads();  // every wave is done with this panel
    store_panel3(pr, tid, sS);  // unconditionally, as in the other forms
    __syncthreads();
  }
}

// dE/dw of the 16 pairs of a wave for one 64-wide k panel, loaded row-coalesced: the
// float32 form covers rows 4 i + l / 16 (i = 0..3) and columns 4 (l % 16) .. + 3 of the
// panel (each load is four full 256-byte row segments); the bfloat16 form covers rows
// 8 i + l / 8 (i = 0..1) and columns 8 (l % 8) .. + 7 (eight full 128-byte row
// segments).  Both edges of a pair are loaded unconditionally (the reverse edge's row
// 2p + 1 exists in the buffer even when the pair has none; rows past the last pair are
// clamped to it) and combined, masked, when the panel is staged.
template <bool BF16>
struct DwRegs {
  static constexpr int N = BF16 ? 2 : 4;  // loads per edge side
  u32x4 a[N], b[N];
};
// row of load i of this lane and its base offset (row 2p of the pair-major buffer)
template <bool BF16>
struct DwRows {
  static constexpr int N = DwRegs<BF16>::N;
  int64_t base[N];
  unsigned ok = 0, two = 0;  // per load: row is a pair; the pair has a reverse edge
  __device__ DwRows(int64_t np, int64_t p_first, const int* __restrict__ pe2, int P, int lane) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int64_t p = p_first + (BF16 ? 8 * i + (lane >> 3) : 4 * i + (lane >> 4));
      const int64_t pc = p < np ? p : np - 1;
      base[i] = 2 * pc * P;
      if (p < np) {
        ok |= 1u << i;
        if (pe2[p] >= 0) two |= 1u << i;
      }
    }
  }
};
template <bool BF16>
__device__ inline int dw_lane_col(int lane) {
  return BF16 ? 8 * (lane & 7) : 4 * (lane & 15);
}
template <bool BF16>
__device__ inline void fetch_dw(const WStore<BF16>* __restrict__ dw, const DwRows<BF16>& rows, int P,
                                int k0, int lane, DwRegs<BF16>& d) {
  constexpr int PER = BF16 ? 8 : 4;
  const int kb = min(k0 + dw_lane_col<BF16>(lane), P - PER);  // P is a multiple of 8
#pragma unroll
  for (int i = 0; i < DwRegs<BF16>::N; ++i) {
    d.a[i] = *reinterpret_cast<const u32x4*>(&dw[rows.base[i] + kb]);
    d.b[i] = *reinterpret_cast<const u32x4*>(&dw[rows.base[i] + P + kb]);
  }
}
// the pair sums of one panel into the wave's LDS tile: float32 rows of stride ZP, or
// bfloat16 rows of stride BP (rounded to nearest even)
template <bool BF16>
__device__ inline void stage_dw(const DwRegs<BF16>& d, const DwRows<BF16>& rows, int P, int k0,
                                int lane, float* Z) {
  const int col = dw_lane_col<BF16>(lane);
  const bool col_ok = k0 + col < P;
#pragma unroll
  for (int i = 0; i < DwRegs<BF16>::N; ++i) {
    const bool valid = col_ok && ((rows.ok >> i) & 1u);
    const bool two = (rows.two >> i) & 1u;
    if constexpr (BF16) {
      const int row = 8 * i + (lane >> 3);
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float fa = __uint_as_float(h ? (d.a[i][e] & 0xffff0000u) : (d.a[i][e] << 16));
          const float fb = __uint_as_float(h ? (d.b[i][e] & 0xffff0000u) : (d.b[i][e] << 16));
          v[2 * e + h] = __float2bfloat16(valid ? (two ? fa + fb : fa) : 0.f);
        }
      }
      *reinterpret_cast<bf16x8*>(reinterpret_cast<__bf16*>(Z) + row * BP + col) = v;
    } else {
      const int row = 4 * i + (lane >> 4);
      const floatx4 fa = __builtin_bit_cast(floatx4, d.a[i]);
      const floatx4 fb = __builtin_bit_cast(floatx4, d.b[i]);
      const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
      *reinterpret_cast<floatx4*>(Z + row * ZP + col) = valid ? (two ? fa + fb : fa) : z;
    }
  }
}

// ------------------------------------------------------------------ backward
// BF16 form (the FP32 form's is the split kernel below)
__global__ __launch_bounds__(256) void k_mlp_fused_bwd(int64_t np, const int* __restrict__ pe1,
                                                        const int* __restrict__ pe2,
                                                        const float* __restrict__ rho,
                                                        const float* __restrict__ Wa,
                                                        const float* __restrict__ Wb,
                                                        const bf16_t* __restrict__ Wcp, int P,
                                                        float c, const bf16_t* __restrict__ dw,
                                                        float* __restrict__ drho, int accumulate) {
  __shared__ float sWa[NBAS * HID];
  __shared__ float sRho[EB * (NBAS + 1)];
  __shared__ float sZ[4][16 * ZP];
  // Wc[j][k-panel]: bfloat16 rows of stride BP
  __shared__ __attribute__((aligned(16))) float sB[2][HID * BP / 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, nullptr, sRho);
  // bfloat16 copies of Wb: the transposed one (hidden-layer recompute) lives in the second
  // panel buffer until the panel loop first fills it, which keeps the block at 48 KB of LDS
  __bf16* sWbT = reinterpret_cast<__bf16*>(sB[1]);
  __shared__ __attribute__((aligned(16))) __bf16 sWbN[HID * BP];
  stage_wb_bf16(Wb, sWbT, sWbN);
  const int r = lane & 15, q = lane >> 4;
  // dE/dw is pair-major: rows 2p (first edge) and 2p + 1 (its reverse, when present)
  const DwRows<true> rows(np, p0 + wave * 16, pe2, P, lane);
  const int npan = (P + HID - 1) / HID;
  PanelRegs wr;
  // dE/dw panels in flight: a ring of RING register sets (RING - 1 panels ahead).  A deeper
  // ring costs the third wave per SIMD (164 registers with 3), and the extra wave hides
  // more than the extra panels did.
  constexpr int RING = 3;
  DwRegs<true> ring[RING];
  fetch_panel(Wcp, 0, npan, tid, wr);
  static_for<RING - 1>([&](auto J) {
    fetch_dw<true>(dw, rows, P, decltype(J)::value * HID, lane, ring[decltype(J)::value]);
  });
  __syncthreads();
  float* Z = sZ[wave];
  // recompute a1 and a2 (accumulator layout)
  floatx4 a1[4], a2[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, a1, lane);
  acc_to_panel(a1, Z, lane, [&](float v, int, int) { return phi(v, c); });
  store_panel(wr, tid, sB[0]);
  __syncthreads();
  zero4(a2);
  panel_bf16(Z, sWbT, a2, lane);
  __syncthreads();  // every wave is done with sWbT before the first panel overwrites it
  // dz2 = (dw[e1] + dw[e2]) Wc^T, contraction over the P radial weights in 64-wide panels
  floatx4 g[4];
  zero4(g);
  // One panel step: the loads ahead (dw of both edges RING - 1 panels ahead, the next Wc
  // panel) are issued first and unconditionally, so they stay in flight across this
  // panel's MFMAs; the panel loop is unrolled by RING so the operand sets rotate through
  // fixed registers (no copies).
  int buf = 0;
  auto step = [&](int jj, auto SLOT) {
    constexpr int rc = decltype(SLOT)::value, rn = (rc + RING - 1) % RING;
    const DwRegs<true>& cur = ring[rc];
    const int k0 = jj * HID;
    fetch_panel(Wcp, jj + 1, npan, tid, wr);
    fetch_dw<true>(dw, rows, P, k0 + (RING - 1) * HID, lane, ring[rn]);
    if (jj < npan) {
      // the pairs' summed dE/dw through the wave's LDS tile into the operand layout
      stage_dw<true>(cur, rows, P, k0, lane, Z);
      const __bf16* sh = reinterpret_cast<const __bf16*>(sB[buf]);
      const __bf16* zh = reinterpret_cast<const __bf16*>(Z);
#pragma unroll
      for (int s = 0; s < HID / 32; ++s) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&zh[r * BP + 32 * s + 8 * q]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sh[(t * 16 + r) * BP + 32 * s + 8 * q]);
          g[t] = mfma32(a, b, g[t]);
        }
      }
    }
    store_panel(wr, tid, sB[buf ^ 1]);
    __syncthreads();
    buf ^= 1;
  };
  for (int j = 0; j < npan; j += RING) {
    static_for<RING>([&](auto J) { step(j + decltype(J)::value, J); });
  }
  // da2 = dz2 * phi'(a2) -> operand panel;  dz1 = da2 Wb^T
  acc_to_panel(g, Z, lane, [&](float v, int t, int rr) { return v * dphi(a2[t][rr], c); });
  __syncthreads();
  floatx4 d1[4];
  zero4(d1);
  panel_bf16(Z, sWbN, d1, lane);
  __syncthreads();
  // da1 = dz1 * phi'(a1) -> operand panel;  drho = da1 Wa^T (8 columns, padded to 16)
  acc_to_panel(d1, Z, lane, [&](float v, int t, int rr) { return v * dphi(a1[t][rr], c); });
  __syncthreads();
  floatx4 dr = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < HID / 4; ++s) {
    const float a = Z[r * ZP + 4 * s + q];
    const float b = (r < NBAS) ? sWa[r * HID + 4 * s + q] : 0.f;
    dr = mfma4(a, b, dr);
  }
  const int col = lane & 15, rq = (lane >> 4) * 4;
  if (col < NBAS) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t p = p0 + wave * 16 + rq + rr;
      if (p < np) {
        const int64_t o = (int64_t)pe1[p] * NBAS + col;
        const float v = dr[rr];
        drho[o] = accumulate ? drho[o] + v : v;
      }
    }
  }
}

// ------------------------------------------------------------------ backward, split form
// The FP32 form's adjoint with dz2 = dw Wc^T in three-part bfloat16 arithmetic (the split
// of the forward above): the pair sums of dE/dw are split as they leave the wave's LDS
// tile, Wc arrives pre-split as [part][j][c] panels, and the six part products with
// i + j <= 2 accumulate in float32.  Float32 matrix cores run at a sixteenth of the
// bfloat16 rate, so six bfloat16 products cost 0.4 of the eight float32 ones they replace.
// One LDS stage for the split panels (two barriers per panel).  The hidden layers stay
// float32 and run after the panel loop: their operands (Wb, Wa, rho) then take the stage's
// memory and a1, a2 are recomputed there, so a block holds 44 KB of LDS and no hidden
// activations during the loop: three blocks per CU, with the registers bounded to match
// (168, no spills, two dE/dw panels ahead).
__global__ __launch_bounds__(256, 3) void k_mlp_fused_bwd_split(int64_t np, const int* __restrict__ pe1,
                                                             const int* __restrict__ pe2,
                                                             const float* __restrict__ rho,
                                                             const float* __restrict__ Wa,
                                                             const float* __restrict__ Wb,
                                                             const bf16_t* __restrict__ Wc3, int P,
                                                             float c, const float* __restrict__ dw,
                                                             float* __restrict__ drho,
                                                             int accumulate) {
  constexpr int kStage = 3 * HID * BP;  // bfloat16 elements of a split-panel stage
  __shared__ float sZ[4][16 * ZP];
  __shared__ __attribute__((aligned(16))) __bf16 sS[kStage];
  static_assert(sizeof(float) * (HID * WP + NBAS * HID + EB * (NBAS + 1)) <= sizeof(__bf16) * kStage,
                "the hidden layers' operands fit the stage");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  const int r = lane & 15, q = lane >> 4;
  // dE/dw is pair-major: rows 2p (first edge) and 2p + 1 (its reverse, when present)
  const DwRows<false> rows(np, p0 + wave * 16, pe2, P, lane);
  const int npan = (P + HID - 1) / HID;
  Panel3Regs pr;
  constexpr int RING = 3;  // dE/dw panels in flight: RING - 1 ahead
  DwRegs<false> ring[RING];
  fetch_panel3(Wc3, 0, npan, tid, pr);
  static_for<RING - 1>([&](auto J) {
    fetch_dw<false>(dw, rows, P, decltype(J)::value * HID, lane, ring[decltype(J)::value]);
  });
  store_panel3(pr, tid, sS);
  __syncthreads();
  float* Z = sZ[wave];
  // dz2 = (dw[e1] + dw[e2]) Wc^T over 64-wide k panels; g[t][rr] = dz2[pair 4 q + rr][16 t + r]
  floatx4 g[4];
  zero4(g);
  auto step = [&](int jj, auto SLOT) {
    constexpr int rc = decltype(SLOT)::value, rn = (rc + RING - 1) % RING;
    const int k0 = jj * HID;
    fetch_panel3(Wc3, jj + 1, npan, tid, pr);
    fetch_dw<false>(dw, rows, P, k0 + (RING - 1) * HID, lane, ring[rn]);
    if (jj < npan) {
      // the wave's own tile, written and then read: LDS operations of one wave complete in
      // order, and the empty asm statements keep the compiler's order
      __asm__ volatile("" ::: "memory");
      stage_dw<false>(ring[rc], rows, P, k0, lane, Z);
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int st = 0; st < HID / 32; ++st) {
        bf16x8 z0, z1, z2;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 h0, h1, h2;
          split3(Z[r * ZP + 32 * st + 8 * q + e], h0, h1, h2);
          z0[e] = h0;
          z1[e] = h1;
          z2[e] = h2;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int off = (16 * t + r) * BP + 32 * st + 8 * q;
          const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(sS + off);
          const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(sS + HID * BP + off);
          const bf16x8 b2 = *reinterpret_cast<const bf16x8*>(sS + 2 * HID * BP + off);
          g[t] = mfma32(z2, b0, g[t]);  // smaller part products first
          g[t] = mfma32(z1, b1, g[t]);
          g[t] = mfma32(z0, b2, g[t]);
          g[t] = mfma32(z1, b0, g[t]);
          g[t] = mfma32(z0, b1, g[t]);
          g[t] = mfma32(z0, b0, g[t]);
        }
      }
      __asm__ volatile("" ::: "memory");
    }
    __syncthreads();  // every wave is done with this panel
    store_panel3(pr, tid, sS);  // unconditionally (a panel past the last is never read)
    __syncthreads();
  };
  for (int j = 0; j < npan; j += RING) {
    static_for<RING>([&](auto J) { step(j + decltype(J)::value, J); });
  }
  // the hidden layers' operands into the stage (every wave is past the last panel)
  float* sWb = reinterpret_cast<float*>(sS);
  float* sWa = sWb + HID * WP;
  float* sRho = sWa + NBAS * HID;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, sWb, sRho);
  __syncthreads();
  // recompute a1 and a2 (accumulator layout)
  floatx4 a1[4], a2[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, a1, lane);
  acc_to_panel(a1, Z, lane, [&](float v, int, int) { return phi(v, c); });
  __syncthreads();
  zero4(a2);
  panel_kn(Z, sWb, a2, lane);
  __syncthreads();
  // da2 = dz2 * phi'(a2) -> operand panel;  dz1 = da2 Wb^T
  acc_to_panel(g, Z, lane, [&](float v, int t, int rr) { return v * dphi(a2[t][rr], c); });
  __syncthreads();
  floatx4 d1[4];
  zero4(d1);
  panel_kn_T(Z, sWb, d1, lane);
  __syncthreads();
  // da1 = dz1 * phi'(a1) -> operand panel;  drho = da1 Wa^T (8 columns, padded to 16)
  acc_to_panel(d1, Z, lane, [&](float v, int t, int rr) { return v * dphi(a1[t][rr], c); });
  __syncthreads();
  floatx4 dr = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < HID / 4; ++s) {
    const float a = Z[r * ZP + 4 * s + q];
    const float b = (r < NBAS) ? sWa[r * HID + 4 * s + q] : 0.f;
    dr = mfma4(a, b, dr);
  }
  const int col = lane & 15, rq = (lane >> 4) * 4;
  if (col < NBAS) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t p = p0 + wave * 16 + rq + rr;
      if (p < np) {
        const int64_t o = (int64_t)pe1[p] * NBAS + col;
        const float v = dr[rr];
        drho[o] = accumulate ? drho[o] + v : v;
      }
    }
  }
}

void launch_mlp_fused_fwd(int64_t np, const int* pe1, const float* rho, const float* Wa,
                          const float* Wb, const bf16_t* Wcp, int P, float c, bf16_t* w,
                          hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  // few pairs: split the output panels over blocks until about 512 blocks run
  const int npan = (P + HID - 1) / HID;
  const unsigned groups = (unsigned)std::max(1, std::min<int>(npan, (int)((512 + grid - 1) / grid)));
  k_mlp_fused_fwd<<<dim3(grid, groups), 256, 0, s>>>(np, pe1, rho, Wa, Wb, Wcp, P, c, w);
}

void launch_mlp_fused_fwd_split(int64_t np, const int* pe1, const float* rho, const float* Wa,
                                const float* Wb, const bf16_t* Wc3, int P, float c, float* w,
                                hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  const int npan = (P + HID - 1) / HID;
  const unsigned groups = (unsigned)std::max(1, std::min<int>(npan, (int)((512 + grid - 1) / grid)));
  k_mlp_fused_fwd_split<<<dim3(grid, groups), 256, 0, s>>>(np, pe1, rho, Wa, Wb, Wc3, P, c, w);
}

void launch_mlp_fused_bwd(int64_t np, const int* pe1, const int* pe2, const float* rho,
                          const float* Wa, const float* Wb, const bf16_t* Wcp, int P, float c,
                          const bf16_t* dw, float* drho, bool accumulate, hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  k_mlp_fused_bwd<<<grid, 256, 0, s>>>(np, pe1, pe2, rho, Wa, Wb, Wcp, P, c, dw, drho,
                                       accumulate ? 1 : 0);
}

void launch_mlp_fused_bwd_split(int64_t np, const int* pe1, const int* pe2, const float* rho,
                                const float* Wa, const float* Wb, const bf16_t* Wc3, int P, float c,
                                const float* dw, float* drho, bool accumulate, hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  k_mlp_fused_bwd_split<<<grid, 256, 0, s>>>(np, pe1, pe2, rho, Wa, Wb, Wc3, P, c, dw, drho,
                                              accumulate ? 1 : 0);
}

}  // namespace sn
