// Fused radial MLP on the matrix cores (float32 and bfloat16 forms).
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
// in LDS once per block and shared by the four waves.  Output panels of w go
// back through LDS so that every store is a full 256-byte row segment.
//
// MFMA layouts (lane l, 16 x 16 tiles):
//   f32 16x16x4  : a = A[l%16][4s + l/16],     b = B[4s + l/16][l%16]
//   bf16 16x16x32: a = A[l%16][32s + 8(l/16) + 0..7], b = B[32s + 8(l/16) + 0..7][l%16]
//   result       : acc[r] = C[4(l/16) + r][l%16]
// LDS strides: operand panels 68 floats, k-major weight panels 80 floats, chosen so
// that the 64 lanes of a fragment read hit distinct banks.
#include "kernels.h"

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
constexpr int TP = 68;   // n-major weight panel stride (floats)
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

// Weight-panel prefetch: each of the 256 threads holds 16 values (4 x 4) of a 64 x 64
// panel in registers while the current panel is being multiplied.  Loads are issued
// unconditionally from clamped addresses (a load under a branch makes the compiler wait
// for it, and for every other load in flight, inside that branch); columns past P are
// zeroed when the panel is staged.
struct PanelRegs {
  float v[16];
};

// Wc panel columns [n0, n0+64) of the forward product, element (k, n) at Wc[k * P + n0 + n]
__device__ inline void fetch_fwd_panel(const float* __restrict__ Wc, int P, int n0, int tid,
                                       PanelRegs& r) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = tid + 256 * j;
    const int k = i / HID, n = i % HID;
    r.v[j] = Wc[(int64_t)k * P + min(n0 + n, P - 1)];
  }
}
template <bool BF16>
__device__ inline void store_fwd_panel(const PanelRegs& r, int tid, int P, int n0, float* sf,
                                       __bf16* sh) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = tid + 256 * j;
    const int k = i / HID, n = i % HID;
    const float v = n0 + n < P ? r.v[j] : 0.f;
    if (BF16) sh[n * BP + k] = __float2bfloat16(v);
    else sf[k * WP + n] = v;
  }
}

// ------------------------------------------------------------------ forward
template <bool BF16>
using WStore = typename std::conditional<BF16, bf16_t, float>::type;

template <bool BF16>
__global__ __launch_bounds__(256) void k_mlp_fused_fwd(int64_t np, const int* __restrict__ pe1,
                                                        const float* __restrict__ rho,
                                                        const float* __restrict__ Wa,
                                                        const float* __restrict__ Wb,
                                                        const float* __restrict__ Wc, int P, float c,
                                                        WStore<BF16>* __restrict__ w) {
  constexpr int PANEL = BF16 ? (HID * BP) / 2 : HID * WP;  // floats per panel buffer
  __shared__ float sWa[NBAS * HID];
  __shared__ float sRho[EB * (NBAS + 1)];
  __shared__ float sZ[4][16 * ZP];
  __shared__ __attribute__((aligned(16))) float sW[2][HID * WP];  // Wb, then Wc panels
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, sW[1], sRho);
  __shared__ __attribute__((aligned(16))) __bf16 sWbT[BF16 ? HID * BP : 8];
  if (BF16) stage_wb_bf16(Wb, sWbT, nullptr);
  PanelRegs pr;
  fetch_fwd_panel(Wc, P, 0, tid, pr);
  __syncthreads();
  float* Z = sZ[wave];
  floatx4 acc[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, acc, lane);
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  store_fwd_panel<BF16>(pr, tid, P, 0, sW[0], reinterpret_cast<__bf16*>(sW[0]));
  __syncthreads();
  zero4(acc);
  if (BF16) panel_bf16(Z, sWbT, acc, lane);
  else panel_kn(Z, sW[1], acc, lane);
  __syncthreads();
  acc_to_panel(acc, Z, lane, [&](float v, int, int) { return phi(v, c); });
  __syncthreads();
  // z2 operand fragments, kept in registers for every output panel
  const int r = lane & 15, q = lane >> 4;
  float za[HID / 4];
  bf16x8 zh[HID / 32];
  if (BF16) {
#pragma unroll
    for (int s = 0; s < HID / 32; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) zh[s][e] = __float2bfloat16(Z[r * ZP + 32 * s + 8 * q + e]);
  } else {
#pragma unroll
    for (int s = 0; s < HID / 4; ++s) za[s] = Z[r * ZP + 4 * s + q];
  }
  (void)PANEL;
  int buf = 0;
  for (int n0 = 0; n0 < P; n0 += HID) {
    fetch_fwd_panel(Wc, P, n0 + HID, tid, pr);  // in flight during the MFMAs (clamped past P)
    __builtin_amdgcn_sched_barrier(0);           // keep the loads ahead of the MFMAs
    const float* sf = sW[buf];
    const __bf16* sh = reinterpret_cast<const __bf16*>(sW[buf]);
    zero4(acc);
    if (BF16) {
#pragma unroll
      for (int s = 0; s < HID / 32; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sh[(t * 16 + r) * BP + 32 * s + 8 * q]);
          acc[t] = mfma32(zh[s], b, acc[t]);
        }
    } else {
#pragma unroll
      for (int s = 0; s < HID / 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mfma4(za[s], sf[(4 * s + q) * WP + t * 16 + r], acc[t]);
    }
    // through the wave's own panel to full-row float4 stores
    acc_to_panel(acc, Z, lane, [](float v, int, int) { return v; });
    // staged unconditionally (the panel past the last is never read): a conditional store
    // would let the compiler sink the panel loads into the branch, after the MFMAs
    store_fwd_panel<BF16>(pr, tid, P, n0 + HID, sW[buf ^ 1], reinterpret_cast<__bf16*>(sW[buf ^ 1]));
    __syncthreads();
    const int c4 = (lane & 15) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int row = (lane >> 4) + 4 * k;
      const int64_t p = p0 + wave * 16 + row;
      if (p < np && n0 + c4 < P) {
        const float* zr = &Z[row * ZP + c4];
        if constexpr (BF16) {  // four bfloat16 values per lane: 128 contiguous bytes per row
          uint2 v;
          v.x = (uint32_t)sstore<bf16_t>(zr[0]).u | ((uint32_t)sstore<bf16_t>(zr[1]).u << 16);
          v.y = (uint32_t)sstore<bf16_t>(zr[2]).u | ((uint32_t)sstore<bf16_t>(zr[3]).u << 16);
          *reinterpret_cast<uint2*>(&w[p * P + n0 + c4]) = v;
        } else {
          *reinterpret_cast<floatx4*>(&w[p * P + n0 + c4]) = floatx4{zr[0], zr[1], zr[2], zr[3]};
        }
      }
    }
    buf ^= 1;
  }
}

// Wc panel for the adjoint: element (j, k) at Wc[j * P + k0 + k] (hidden row j)
__device__ inline void fetch_bwd_panel(const float* __restrict__ Wc, int P, int k0, int tid,
                                       PanelRegs& r) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = tid + 256 * j;
    const int jj = i / HID, k = i % HID;
    r.v[j] = Wc[(int64_t)jj * P + min(k0 + k, P - 1)];
  }
}
template <bool BF16>
__device__ inline void store_bwd_panel(const PanelRegs& r, int tid, int P, int k0, float* sf,
                                       __bf16* sh) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int i = tid + 256 * j;
    const int jj = i / HID, k = i % HID;
    const float v = k0 + k < P ? r.v[j] : 0.f;
    if (BF16) sh[jj * BP + k] = __float2bfloat16(v);
    else sf[jj * TP + k] = v;
  }
}

// dw operand of one lane for a 64-wide k panel, both edges of the pair loaded separately
// and unconditionally (clamped addresses; a missing reverse edge reads the first row
// again) and combined when the panel is used.  float32 form: lane group q covers
// k = 16 u + 4 q + 0..3; bfloat16 form: k = 32 (u / 2) + 8 q + 4 (u % 2) + 0..3, the order
// of the 16x16x32 operand.
template <bool BF16>
struct DwRegs;
template <>
struct DwRegs<false> {  // float32 dE/dw: 16 values per edge row per panel
  floatx4 a[HID / 16], b[HID / 16];
};
template <>
struct DwRegs<true> {  // bfloat16 dE/dw: 2 x 8 values per edge row per panel
  uint4 a[HID / 32], b[HID / 32];
};
__device__ inline int dw_col(int k0, int u, int q) { return k0 + 16 * u + 4 * q; }
__device__ inline int dw_col16(int k0, int s, int q) { return k0 + 32 * s + 8 * q; }

__device__ inline void fetch_dw(const float* __restrict__ dw, int64_t r1, int64_t r2, int P, int k0,
                                int q, DwRegs<false>& d) {
#pragma unroll
  for (int u = 0; u < HID / 16; ++u) {
    const int kb = min(dw_col(k0, u, q), P - 4);  // P is a multiple of 4
    d.a[u] = *reinterpret_cast<const floatx4*>(&dw[r1 + kb]);
    d.b[u] = *reinterpret_cast<const floatx4*>(&dw[r2 + kb]);
  }
}
__device__ inline void fetch_dw(const bf16_t* __restrict__ dw, int64_t r1, int64_t r2, int P,
                                int k0, int q, DwRegs<true>& d) {
#pragma unroll
  for (int s = 0; s < HID / 32; ++s) {
    const int kb = min(dw_col16(k0, s, q), P - 8);  // P is a multiple of 8
    d.a[s] = *reinterpret_cast<const uint4*>(&dw[r1 + kb]);
    d.b[s] = *reinterpret_cast<const uint4*>(&dw[r2 + kb]);
  }
}
__device__ inline floatx4 dw_value(const DwRegs<false>& d, int u, bool row_ok, bool has2, int P,
                                   int k0, int q) {
  const floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
  if (!row_ok || dw_col(k0, u, q) >= P) return z;
  return has2 ? d.a[u] + d.b[u] : d.a[u];
}
// operand of the 16x16x32 product: the pair's summed dE/dw at k = 32 s + 8 q + 0..7
__device__ inline bf16x8 dw_value16(const DwRegs<true>& d, int s, bool row_ok, bool has2, int P,
                                    int k0, int q) {
  const bool valid = row_ok && dw_col16(k0, s, q) < P;
  const uint32_t av[4] = {d.a[s].x, d.a[s].y, d.a[s].z, d.a[s].w};
  const uint32_t bv[4] = {d.b[s].x, d.b[s].y, d.b[s].z, d.b[s].w};
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float fa = __uint_as_float(h ? (av[i] & 0xffff0000u) : (av[i] << 16));
      const float fb = __uint_as_float(h ? (bv[i] & 0xffff0000u) : (bv[i] << 16));
      const float f = valid ? (has2 ? fa + fb : fa) : 0.f;
      r[2 * i + h] = __float2bfloat16(f);
    }
  }
  return r;
}

// ------------------------------------------------------------------ backward
template <bool BF16>
__global__ __launch_bounds__(256) void k_mlp_fused_bwd(int64_t np, const int* __restrict__ pe1,
                                                        const int* __restrict__ pe2,
                                                        const float* __restrict__ rho,
                                                        const float* __restrict__ Wa,
                                                        const float* __restrict__ Wb,
                                                        const float* __restrict__ Wc, int P, float c,
                                                        const WStore<BF16>* __restrict__ dw,
                                                        float* __restrict__ drho, int accumulate) {
  __shared__ float sWa[NBAS * HID];
  __shared__ float sWb[BF16 ? 4 : HID * WP];  // float32 form only (bfloat16 copies below)
  __shared__ float sRho[EB * (NBAS + 1)];
  __shared__ float sZ[4][16 * ZP];
  // Wc[j][k-panel]: float32 rows of stride TP, or bfloat16 rows of stride BP
  __shared__ __attribute__((aligned(16))) float sB[2][BF16 ? HID * BP / 2 : HID * TP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * EB;
  stage_common(np, p0, pe1, rho, Wa, Wb, sWa, BF16 ? nullptr : sWb, sRho);
  __shared__ __attribute__((aligned(16))) __bf16 sWbT[BF16 ? HID * BP : 8];
  __shared__ __attribute__((aligned(16))) __bf16 sWbN[BF16 ? HID * BP : 8];
  if (BF16) stage_wb_bf16(Wb, sWbT, sWbN);
  const int r = lane & 15, q = lane >> 4;
  const int64_t pr = p0 + wave * 16 + r;
  const bool row_ok = pr < np;
  // dE/dw is pair-major: rows 2p (first edge) and 2p + 1 (its reverse, when present)
  const int64_t r1 = row_ok ? 2 * pr * P : 0;
  const bool has2 = row_ok && pe2[pr] >= 0;
  const int64_t r2 = has2 ? r1 + P : r1;
  PanelRegs wr;
  // dE/dw panels in flight: a ring of RING register sets (RING - 1 panels ahead); the
  // bfloat16 operands are small and the matrix cores fast, so that form looks further ahead
  constexpr int RING = BF16 ? 4 : 2;
  DwRegs<BF16> ring[RING];
  fetch_bwd_panel(Wc, P, 0, tid, wr);
  static_for<RING - 1>([&](auto J) {
    fetch_dw(dw, r1, r2, P, decltype(J)::value * HID, q, ring[decltype(J)::value]);
  });
  __syncthreads();
  float* Z = sZ[wave];
  // recompute a1 and a2 (accumulator layout)
  floatx4 a1[4], a2[4];
  first_layer(sRho + wave * 16 * (NBAS + 1), sWa, a1, lane);
  acc_to_panel(a1, Z, lane, [&](float v, int, int) { return phi(v, c); });
  store_bwd_panel<BF16>(wr, tid, P, 0, sB[0], reinterpret_cast<__bf16*>(sB[0]));
  __syncthreads();
  zero4(a2);
  if (BF16) panel_bf16(Z, sWbT, a2, lane);
  else panel_kn(Z, sWb, a2, lane);
  // dz2 = (dw[e1] + dw[e2]) Wc^T, contraction over the P radial weights in 64-wide panels
  floatx4 g[4];
  zero4(g);
  // One panel step: the loads ahead (dw of both edges RING - 1 panels ahead, the next Wc
  // panel) are issued first and unconditionally, so they stay in flight across this
  // panel's MFMAs; the panel loop is unrolled by RING so the operand sets rotate through
  // fixed registers (no copies).
  const int npan = (P + HID - 1) / HID;
  int buf = 0;
  auto step = [&](int jj, auto SLOT) {
    constexpr int rc = decltype(SLOT)::value, rn = (rc + RING - 1) % RING;
    const DwRegs<BF16>& cur = ring[rc];
    const int k0 = jj * HID;
    fetch_bwd_panel(Wc, P, k0 + HID, tid, wr);
    fetch_dw(dw, r1, r2, P, k0 + (RING - 1) * HID, q, ring[rn]);
    if (jj < npan) {
      if constexpr (BF16) {
        const __bf16* sh = reinterpret_cast<const __bf16*>(sB[buf]);
#pragma unroll
        for (int s = 0; s < HID / 32; ++s) {
          const bf16x8 a = dw_value16(cur, s, row_ok, has2, P, k0, q);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sh[(t * 16 + r) * BP + 32 * s + 8 * q]);
            g[t] = mfma32(a, b, g[t]);
          }
        }
      } else {
        const float* sf = sB[buf];
#pragma unroll
        for (int u = 0; u < HID / 16; ++u) {
          const floatx4 av = dw_value(cur, u, row_ok, has2, P, k0, q);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const floatx4 bv =
                *reinterpret_cast<const floatx4*>(&sf[(t * 16 + r) * TP + 16 * u + 4 * q]);
#pragma unroll
            for (int s = 0; s < 4; ++s) g[t] = mfma4(av[s], bv[s], g[t]);
          }
        }
      }
    }
    store_bwd_panel<BF16>(wr, tid, P, k0 + HID, sB[buf ^ 1], reinterpret_cast<__bf16*>(sB[buf ^ 1]));
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
  if (BF16) panel_bf16(Z, sWbN, d1, lane);
  else panel_kn_T(Z, sWb, d1, lane);
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

template <typename WS>
void launch_mlp_fused_fwd(int64_t np, const int* pe1, const float* rho, const float* Wa,
                          const float* Wb, const float* Wc, int P, float c, WS* w, hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  constexpr bool BF16 = std::is_same<WS, bf16_t>::value;
  k_mlp_fused_fwd<BF16><<<grid, 256, 0, s>>>(np, pe1, rho, Wa, Wb, Wc, P, c, w);
}

template <typename WS>
void launch_mlp_fused_bwd(int64_t np, const int* pe1, const int* pe2, const float* rho,
                          const float* Wa, const float* Wb, const float* Wc, int P, float c,
                          const WS* dw, float* drho, bool accumulate, hipStream_t s) {
  if (np <= 0) return;
  const unsigned grid = (unsigned)((np + EB - 1) / EB);
  constexpr bool BF16 = std::is_same<WS, bf16_t>::value;
  k_mlp_fused_bwd<BF16><<<grid, 256, 0, s>>>(np, pe1, pe2, rho, Wa, Wb, Wc, P, c, dw, drho,
                                             accumulate ? 1 : 0);
}

template void launch_mlp_fused_fwd<float>(int64_t, const int*, const float*, const float*,
                                          const float*, const float*, int, float, float*,
                                          hipStream_t);
template void launch_mlp_fused_fwd<bf16_t>(int64_t, const int*, const float*, const float*,
                                           const float*, const float*, int, float, bf16_t*,
                                           hipStream_t);
template void launch_mlp_fused_bwd<float>(int64_t, const int*, const int*, const float*,
                                          const float*, const float*, const float*, int, float,
                                          const float*, float*, bool, hipStream_t);
template void launch_mlp_fused_bwd<bf16_t>(int64_t, const int*, const int*, const float*,
                                           const float*, const float*, const float*, int, float,
                                           const bf16_t*, float*, bool, hipStream_t);

}  // namespace sn
