// Matrix-core GEMM for the float32 and bfloat16 forms (gfx950 MFMA).
//
// C[M x N] (=|+=) alpha * A[M x K] op(B) with float32 accumulation; A and C rows
// are addressed through RowMap (so the same kernel serves the per-degree channel
// mixing on interleaved feature rows and the radial-MLP output layer on plain
// edge rows).  64 x 64 block tile, four waves in a 2 x 2 arrangement, each
// wave owning a 32 x 32 sub-tile = 2 x 2 MFMA tiles of 16 x 16:
//   float32 : v_mfma_f32_16x16x4_f32, k-step 16 staged in LDS
//   bfloat16: v_mfma_f32_16x16x32_bf16, k-step 32 staged in LDS (operands rounded
//             to bfloat16 with round-to-nearest-even when staged)
// MFMA 16 x 16 operand layout (lane l): A[row l%16][k-group l/16], B[k-group l/16]
// [col l%16]; result lane l holds rows 4*(l/16) + r (r = 0..3) of column l%16.
// Blocks are mapped XCD-contiguously: consecutive tiles of one row panel land on
// the same XCD, so the A panel is read once per XCD L2.
#include "kernels.h"

#include <type_traits>

namespace sn {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MT = 64;  // block tile rows / cols

template <typename T>
__device__ inline float to_float(T v) { return (float)v; }

__device__ inline __bf16 to_bf16(float v) {
  return __float2bfloat16(v);
}

template <typename TA, typename TB, typename TC, bool BT, bool BF16>
__global__ __launch_bounds__(256) void k_gemm_mfma(int64_t M, int N, int K, const TA* __restrict__ A,
                                                    RowMap am, const TB* __restrict__ B, int ldb,
                                                    TC* __restrict__ C, RowMap cm, float alpha,
                                                    int accumulate, int nbn, int64_t ntiles,
                                                    int64_t chunk) {
  constexpr int BK = BF16 ? 32 : 16;
  constexpr int PAD = BF16 ? 8 : 1;
  using ST = typename std::conditional<BF16, __bf16, float>::type;
  __shared__ __attribute__((aligned(16))) ST As[MT][BK + PAD];
  __shared__ __attribute__((aligned(16))) ST Bs[MT][BK + PAD];  // stored [n][k]
  // XCD-contiguous tile order
  const int64_t p = blockIdx.x;
  const int64_t tile = (p % 8) * chunk + p / 8;
  if (tile >= ntiles) return;
  const int64_t mb = tile / nbn;
  const int nbk = (int)(tile % nbn);
  const int64_t m0 = mb * MT;
  const int n0 = nbk * MT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // global -> LDS assignment
  constexpr int EPT = BK / 4;             // elements per thread along k
  const int lr = tid >> 2;                 // row (A) or n (B^T) 0..63
  const int lk = (tid & 3) * EPT;          // first k
  const int64_t arow_g = m0 + lr;
  const bool arow_ok = arow_g < M;
  const int64_t arow = arow_ok ? am(arow_g) : 0;
  // non-transposed B: thread covers k = tid / (64 / (BK/4))...: use (k, 4 consecutive n)
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = k0 + lk + e;
      float v = (arow_ok && k < K) ? to_float(A[arow + k]) : 0.f;
      As[lr][lk + e] = (ST)v;
    }
    if (BT) {
      const int n = n0 + lr;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int k = k0 + lk + e;
        float v = (n < N && k < K) ? to_float(B[(int64_t)n * ldb + k]) : 0.f;
        Bs[lr][lk + e] = (ST)v;
      }
    } else {
      // B is K x N row-major: thread loads EPT values of one k along n
      constexpr int TPR = MT / 4;  // threads per k-row when each loads 4 n
      for (int idx = tid; idx < BK * (MT / 4); idx += 256) {
        const int kk = idx / TPR;
        const int nn = (idx % TPR) * 4;
        const int k = k0 + kk;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int n = n0 + nn + e;
          float v = (k < K && n < N) ? to_float(B[(int64_t)k * ldb + n]) : 0.f;
          Bs[nn + e][kk] = (ST)v;
        }
      }
    }
    __syncthreads();
    if constexpr (BF16) {
      const int r = lane & 15, kq = (lane >> 4) * 8;
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8*>(&As[wr + i * 16 + r][kq]);
        b[i] = *reinterpret_cast<const bf16x8*>(&Bs[wc + i * 16 + r][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
      const int r = lane & 15, kq = lane >> 4;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i] = As[wr + i * 16 + r][kk + kq];
          b[i] = Bs[wc + i * 16 + r][kk + kq];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int col_l = lane & 15, row_q = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc + j * 16 + col_l;
      if (col >= N) continue;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t row = m0 + wr + i * 16 + row_q + rr;
        if (row >= M) continue;
        TC* c = C + cm(row) + col;
        float v = alpha * acc[i][j][rr];
        *c = accumulate ? (TC)((float)*c + v) : (TC)v;
      }
    }
}

template <typename TA, typename TB, typename TC>
void launch_gemm_mfma(int64_t M, int N, int K, const TA* A, RowMap am, const TB* B, int ldb, bool bt,
                      TC* C, RowMap cm, float alpha, bool accumulate, bool bf16, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const int nbn = (N + MT - 1) / MT;
  const int64_t nbm = (M + MT - 1) / MT;
  const int64_t ntiles = nbm * nbn;
  const int64_t chunk = (ntiles + 7) / 8;
  const unsigned grid = (unsigned)(chunk * 8);
#define SN_L(BTV, BFV)                                                                       \
  k_gemm_mfma<TA, TB, TC, BTV, BFV><<<grid, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm, alpha, \
                                                         accumulate ? 1 : 0, nbn, ntiles, chunk)
  if (bt) {
    if (bf16) SN_L(true, true); else SN_L(true, false);
  } else {
    if (bf16) SN_L(false, true); else SN_L(false, false);
  }
#undef SN_L
}

#define SN_MFMA_INST(TA, TB, TC)                                                               \
  template void launch_gemm_mfma<TA, TB, TC>(int64_t, int, int, const TA*, RowMap, const TB*,   \
                                             int, bool, TC*, RowMap, float, bool, bool,         \
                                             hipStream_t);
SN_MFMA_INST(float, float, float)
SN_MFMA_INST(float, float, double)
SN_MFMA_INST(double, float, float)
SN_MFMA_INST(double, float, double)
SN_MFMA_INST(double, double, float)
SN_MFMA_INST(double, double, double)
#undef SN_MFMA_INST

}  // namespace sn
