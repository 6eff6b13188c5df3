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
// [col l%16]; result lane l holds rows 4*(l/16) + r (r = 0..3) of column l%16.  The
// vector-load kernels (k_gemm_mfma_v, _vg) issue each product transposed (the B fragment
// in the A slot), so lane l holds columns 4*(l/16) + r of row l%16 and writes them as one
// vector store (element by element where a C row start is not aligned for it): step
// -0.4 ms FP32, -0.3 ms BF16 against four scattered scalar stores per lane and tile.
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
template <>
__device__ inline float to_float<bf16_t>(bf16_t v) { return sload(v); }

// C element update (= v or += v) in the output type
template <typename TC>
__device__ inline void put(TC* c, float v, int accumulate) {
  *c = accumulate ? (TC)(*c + (TC)v) : (TC)v;
}
template <>
__device__ inline void put<bf16_t>(bf16_t* c, float v, int accumulate) {
  *c = sstore<bf16_t>(accumulate ? sload(*c) + v : v);
}

// four consecutive C elements (= or +=), as one vector access where the row is aligned
// for it (cvec), else element by element; each element rounds as put() does
template <typename TC>
__device__ inline void put4(TC* c, float alpha, floatx4 v, int accumulate, int cvec) {
#pragma unroll
  for (int e = 0; e < 4; ++e) put(c + e, alpha * v[e], accumulate);
}
template <>
__device__ inline void put4<float>(float* c, float alpha, floatx4 v, int accumulate, int cvec) {
  if (cvec) {
    floatx4 x = alpha * v;
    if (accumulate) x += *reinterpret_cast<const floatx4*>(c);
    *reinterpret_cast<floatx4*>(c) = x;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) put(c + e, alpha * v[e], accumulate);
  }
}
template <>
__device__ inline void put4<bf16_t>(bf16_t* c, float alpha, floatx4 v, int accumulate, int cvec) {
  if (cvec) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    u32x2 old = accumulate ? *reinterpret_cast<const u32x2*>(c) : u32x2{0u, 0u};
    u32x2 out;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float lo = alpha * v[2 * h], hi = alpha * v[2 * h + 1];
      if (accumulate) {
        lo = __uint_as_float(old[h] << 16) + lo;
        hi = __uint_as_float(old[h] & 0xffff0000u) + hi;
      }
      out[h] = (uint32_t)sstore<bf16_t>(lo).u | ((uint32_t)sstore<bf16_t>(hi).u << 16);
    }
    *reinterpret_cast<u32x2*>(c) = out;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) put(c + e, alpha * v[e], accumulate);
  }
}
template <>
__device__ inline void put4<double>(double* c, float alpha, floatx4 v, int accumulate, int cvec) {
  if (cvec) {
    typedef double doublex2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      doublex2 x = {(double)(alpha * v[2 * h]), (double)(alpha * v[2 * h + 1])};
      if (accumulate) {
        const doublex2 o = reinterpret_cast<const doublex2*>(c)[h];
        x = doublex2{o[0] + x[0], o[1] + x[1]};
      }
      reinterpret_cast<doublex2*>(c)[h] = x;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) put(c + e, alpha * v[e], accumulate);
  }
}

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
        put(C + cm(row) + col, alpha * acc[i][j][rr], accumulate);
      }
    }
}

// ------------------------------------------------------------------ vector-load variant
// Same contraction for aligned operands (rows, leading dimensions and offsets multiples of
// 16 bytes, K and N multiples of 8): k-slabs of 32 loaded with 16-byte vector loads one
// slab ahead into registers, staged in double-buffered LDS (one barrier per slab), and
// block tiles of 64 x BN with BN = 32 for narrow outputs.
template <typename T>
__device__ inline void ld4(const T* p, float (&v)[4]);
template <>
__device__ inline void ld4<float>(const float* p, float (&v)[4]) {
  const floatx4 a = *reinterpret_cast<const floatx4*>(p);
  v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
}
template <>
__device__ inline void ld4<bf16_t>(const bf16_t* p, float (&v)[4]) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 a = *reinterpret_cast<const u32x2*>(p);
  v[0] = __uint_as_float(a[0] << 16); v[1] = __uint_as_float(a[0] & 0xffff0000u);
  v[2] = __uint_as_float(a[1] << 16); v[3] = __uint_as_float(a[1] & 0xffff0000u);
}
template <>
__device__ inline void ld4<double>(const double* p, float (&v)[4]) {
  typedef double doublex2 __attribute__((ext_vector_type(2)));
  const doublex2 a = *reinterpret_cast<const doublex2*>(p);
  const doublex2 b = *reinterpret_cast<const doublex2*>(p + 2);
  v[0] = (float)a[0]; v[1] = (float)a[1]; v[2] = (float)b[0]; v[3] = (float)b[1];
}

// NBUF LDS stages: 2 (one barrier per slab) or 1 (two barriers per slab, half the LDS, so
// twice the resident blocks per CU; the next slab is in registers either way)
template <bool BF16, int BN, int BK, int NBUF = 2>
struct VTileLds {
  static constexpr int BM = 64;
  static constexpr int SP = BF16 ? BK + 8 : BK + 4;  // LDS row stride (16-byte aligned rows)
  using ST = typename std::conditional<BF16, __bf16, float>::type;
  ST a[NBUF][BM][SP];
  ST b[NBUF][BN][SP];  // stored [n][k]
};

// one 64 x BN output tile (rows m0.., columns n0..) of C (=|+=) alpha * A op(B) in k-slabs of
// BK (a multiple of 32); each output element accumulates over k in the same order for any
// slab width.
template <typename TA, typename TB, typename TC, bool BT, bool BF16, int BN, int BK, int NBUF>
__device__ inline void gemm_v_tile(int64_t M, int N, int K, const TA* __restrict__ A, RowMap am,
                                   const TB* __restrict__ B, int ldb, TC* __restrict__ C, RowMap cm,
                                   float alpha, int accumulate, int cvec, int64_t m0, int n0,
                                   VTileLds<BF16, BN, BK, NBUF>& L) {
  using ST = typename VTileLds<BF16, BN, BK, NBUF>::ST;
  auto& As = L.a;
  auto& Bs = L.b;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int TM = BN == 64 ? 2 : 1;  // 16-row tiles per wave
  const int wr = BN == 64 ? (wave >> 1) * 32 : wave * 16;
  const int wc = BN == 64 ? (wave & 1) * 32 : 0;
  floatx4 acc[TM][2];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // A: thread covers row tid/4, k = AE (tid%4) .. + AE - 1
  constexpr int AE = BK / 4;
  const int ar = tid >> 2, ak = (tid & 3) * AE;
  const bool a_ok = m0 + ar < M;
  const TA* a_src = A + (a_ok ? am(m0 + ar) : 0) + ak;
  // B: BN*BK/256 elements per thread
  constexpr int BE = BN * BK / 256;  // 4, 8 or 16
  int bn, bk;
  if (BT) {  // B[n][k]: thread covers n, BE consecutive k
    bn = tid / (BK / BE);
    bk = (tid % (BK / BE)) * BE;
  } else {   // B[k][n]: thread covers k, BE consecutive n
    bk = tid / (BN / BE);
    bn = (tid % (BN / BE)) * BE;
  }
  const TB* b_src = BT ? B + (int64_t)(n0 + bn) * ldb + bk : B + (int64_t)bk * ldb + n0 + bn;
  float ra[AE], rb[BE];
  // K and N are multiples of 8, so each group of (up to) 8 values is all in or all out
  auto fetch = [&](int k0) {
    float t[4];
#pragma unroll
    for (int h = 0; h < AE; h += 8) {
      if (a_ok && k0 + ak + h < K) {
        ld4<TA>(a_src + k0 + h, t);
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[h + e] = t[e];
        ld4<TA>(a_src + k0 + h + 4, t);
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[h + 4 + e] = t[e];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[h + e] = 0.f;
      }
    }
    constexpr int CH = BE < 8 ? BE : 8;
#pragma unroll
    for (int h = 0; h < BE; h += CH) {
      const bool in = BT ? (n0 + bn < N && k0 + bk + h < K) : (k0 + bk < K && n0 + bn + h < N);
      if (in) {
        const TB* q = (BT ? b_src + k0 : b_src + (int64_t)k0 * ldb) + h;
#pragma unroll
        for (int e = 0; e < CH; e += 4) {
          ld4<TB>(q + e, t);
#pragma unroll
          for (int f = 0; f < 4; ++f) rb[h + e + f] = t[f];
        }
      } else {
#pragma unroll
        for (int e = 0; e < CH; ++e) rb[h + e] = 0.f;
      }
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) As[buf][ar][ak + e] = (ST)ra[e];
    if (BT) {
#pragma unroll
      for (int e = 0; e < BE; ++e) Bs[buf][bn][bk + e] = (ST)rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < BE; ++e) Bs[buf][bn + e][bk] = (ST)rb[e];
    }
  };
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    stage(buf);
    __syncthreads();
    if (k0 + BK < K) fetch(k0 + BK);
    if constexpr (BF16) {
      const int r = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
      for (int kb = 0; kb < BK; kb += 32) {
        bf16x8 a[TM], b[2];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wr + i * 16 + r][kb + kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
          b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wc + j * 16 + r][kb + kq]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[i][j], 0, 0, 0);
      }
    } else {
      const int r = lane & 15, kq = lane >> 4;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[TM], b[2];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[buf][wr + i * 16 + r][kk + kq];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[buf][wc + j * 16 + r][kk + kq];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[j], a[i], acc[i][j], 0, 0, 0);
      }
    }
    if (NBUF == 1) __syncthreads();  // every wave is done with the stage before it is refilled
    buf ^= NBUF - 1;
  }
  // the products ran transposed (B fragment in the A slot), so lane l holds row l % 16 of a
  // tile and its four consecutive columns 4 (l / 16) .. + 3: one vector store per tile
  const int row_l = lane & 15, col_q = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc + j * 16 + col_q;
      const int64_t row = m0 + wr + i * 16 + row_l;
      if (col >= N || row >= M) continue;  // N % 8 == 0: the four columns are all in
      put4(C + cm(row) + col, alpha, acc[i][j], accumulate, cvec);
    }
}

template <typename TA, typename TB, typename TC, bool BT, bool BF16, int BN>
__global__ __launch_bounds__(256) void k_gemm_mfma_v(int64_t M, int N, int K, const TA* __restrict__ A,
                                                      RowMap am, const TB* __restrict__ B, int ldb,
                                                      TC* __restrict__ C, RowMap cm, float alpha,
                                                      int accumulate, int cvec, int nbn,
                                                      int64_t ntiles, int64_t chunk) {
  __shared__ __attribute__((aligned(16))) VTileLds<BF16, BN, 32, 1> lds;
  const int64_t p = blockIdx.x;
  const int64_t tile = (p % 8) * chunk + p / 8;
  if (tile >= ntiles) return;
  gemm_v_tile<TA, TB, TC, BT, BF16, BN, 32, 1>(M, N, K, A, am, B, ldb, C, cm, alpha, accumulate, cvec,
                                               (tile / nbn) * 64, (int)(tile % nbn) * BN, lds);
}

// grouped launch: problem q owns tiles [tile0[q], tile0[q + 1])
template <typename TA, typename TB, typename TC>
struct GemmGroupArgs {
  GemmDesc<TA, TB, TC> d[kMaxGemmGroup];
  int64_t tile0[kMaxGemmGroup + 1];
  int nbn[kMaxGemmGroup];
  int cvec[kMaxGemmGroup];
  int n;
  int64_t chunk;
};

template <typename TA, typename TB, typename TC, bool BT, bool BF16, int BN>
__global__ __launch_bounds__(256) void k_gemm_mfma_vg(GemmGroupArgs<TA, TB, TC> g) {
  __shared__ __attribute__((aligned(16))) VTileLds<BF16, BN, 32, 2> lds;
  const int64_t p = blockIdx.x;
  const int64_t tile = (p % 8) * g.chunk + p / 8;
  if (tile >= g.tile0[g.n]) return;
  int q = 0;
  while (q + 1 < g.n && tile >= g.tile0[q + 1]) ++q;
  const GemmDesc<TA, TB, TC>& d = g.d[q];
  const int64_t t = tile - g.tile0[q];
  gemm_v_tile<TA, TB, TC, BT, BF16, BN, 32, 2>(d.M, d.N, d.K, d.A, d.am, d.B, d.ldb, d.C, d.cm,
                                            (float)d.alpha, d.accumulate, g.cvec[q], (t / g.nbn[q]) * 64,
                                            (int)(t % g.nbn[q]) * BN, lds);
}

template <typename T>
static bool aligned16(const T* p, int64_t a, int64_t b, int64_t c) {
  constexpr int64_t q = 16 / sizeof(T);
  return ((uintptr_t)p % 16 == 0) && a % q == 0 && b % q == 0 && c % q == 0;
}

// whether every C row start suits put4's vector access (16 bytes of float, 8 of bfloat16,
// 16 per double pair)
template <typename TC>
static int c_vector_ok(const TC* C, RowMap cm) {
  constexpr int64_t q = std::is_same<TC, double>::value ? 2 : 4;
  constexpr uintptr_t al = std::is_same<TC, bf16_t>::value ? 8 : 16;
  return ((uintptr_t)C % al == 0) && cm.stride % q == 0 && cm.off % q == 0 &&
         (cm.nm <= 1 || cm.ld % q == 0);
}

template <typename TA, typename TB, typename TC>
void launch_gemm_mfma(int64_t M, int N, int K, const TA* A, RowMap am, const TB* B, int ldb, bool bt,
                      TC* C, RowMap cm, float alpha, bool accumulate, bool bf16, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const bool vec = K % 8 == 0 && N % 8 == 0 && aligned16(A, am.stride, am.off, am.nm > 1 ? am.ld : 0) &&
                   aligned16(B, ldb, 0, 0);
  if (vec) {
    const int bn = N <= 32 ? 32 : 64;
    const int nbn = (N + bn - 1) / bn;
    const int64_t ntiles = ((M + 63) / 64) * nbn;
    const int64_t chunk = (ntiles + 7) / 8;
    const unsigned grid = (unsigned)(chunk * 8);
    const int accv = accumulate ? 1 : 0, cv = c_vector_ok(C, cm);
#define SN_V(BTV, BFV, BNV)                                                                      \
  k_gemm_mfma_v<TA, TB, TC, BTV, BFV, BNV><<<grid, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm,    \
                                                               alpha, accv, cv, nbn, ntiles, chunk)
    if (bn == 32) {
      if (bt) { if (bf16) SN_V(true, true, 32); else SN_V(true, false, 32); }
      else { if (bf16) SN_V(false, true, 32); else SN_V(false, false, 32); }
    } else {
      if (bt) { if (bf16) SN_V(true, true, 64); else SN_V(true, false, 64); }
      else { if (bf16) SN_V(false, true, 64); else SN_V(false, false, 64); }
    }
#undef SN_V
    return;
  }
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

template <typename TA, typename TB, typename TC>
void launch_gemm_mfma_group(int n, const GemmDesc<TA, TB, TC>* d, bool bt, bool bf16, hipStream_t s) {
  GemmGroupArgs<TA, TB, TC> g{};
  bool vec = n <= kMaxGemmGroup;
  bool narrow = true;
  for (int q = 0; q < n && vec; ++q) {
    if (d[q].M <= 0 || d[q].N <= 0) continue;
    vec = d[q].K % 8 == 0 && d[q].N % 8 == 0 &&
          aligned16(d[q].A, d[q].am.stride, d[q].am.off, d[q].am.nm > 1 ? d[q].am.ld : 0) &&
          aligned16(d[q].B, d[q].ldb, 0, 0);
    narrow = narrow && d[q].N <= 32;
    g.d[g.n++] = d[q];
  }
  int64_t tiles = 0;
  for (int q = 0; q < g.n; ++q)
    tiles += ((g.d[q].M + 63) / 64) * ((g.d[q].N + (narrow ? 31 : 63)) / (narrow ? 32 : 64));
  // grouping pays where the problems are too small to fill the chip one at a time; larger
  // ones keep their own launches (and the overlap with the second stream they were tuned for)
  if (!vec || g.n <= 1 || tiles > kGroupMaxTiles) {  // one launch per problem
    for (int q = 0; q < n; ++q)
      launch_gemm_mfma<TA, TB, TC>(d[q].M, d[q].N, d[q].K, d[q].A, d[q].am, d[q].B, d[q].ldb, bt,
                                   d[q].C, d[q].cm, (float)d[q].alpha, d[q].accumulate != 0, bf16,
                                   s);
    return;
  }
  const int bn = narrow ? 32 : 64;
  g.tile0[0] = 0;
  for (int q = 0; q < g.n; ++q) {
    g.nbn[q] = (g.d[q].N + bn - 1) / bn;
    g.cvec[q] = c_vector_ok(g.d[q].C, g.d[q].cm);
    g.tile0[q + 1] = g.tile0[q] + ((g.d[q].M + 63) / 64) * g.nbn[q];
  }
  g.chunk = (g.tile0[g.n] + 7) / 8;
  const unsigned grid = (unsigned)(g.chunk * 8);
#define SN_G(BTV, BFV, BNV) k_gemm_mfma_vg<TA, TB, TC, BTV, BFV, BNV><<<grid, 256, 0, s>>>(g)
  if (bn == 32) {
    if (bt) { if (bf16) SN_G(true, true, 32); else SN_G(true, false, 32); }
    else { if (bf16) SN_G(false, true, 32); else SN_G(false, false, 32); }
  } else {
    if (bt) { if (bf16) SN_G(true, true, 64); else SN_G(true, false, 64); }
    else { if (bf16) SN_G(false, true, 64); else SN_G(false, false, 64); }
  }
#undef SN_G
}

#define SN_MFMA_INST(TA, TB, TC)                                                               \
  template void launch_gemm_mfma<TA, TB, TC>(int64_t, int, int, const TA*, RowMap, const TB*,   \
                                             int, bool, TC*, RowMap, float, bool, bool,         \
                                             hipStream_t);                                     \
  template void launch_gemm_mfma_group<TA, TB, TC>(int, const GemmDesc<TA, TB, TC>*, bool, bool, \
                                                   hipStream_t);
SN_MFMA_INST(float, float, float)
SN_MFMA_INST(float, float, double)
SN_MFMA_INST(double, float, float)
SN_MFMA_INST(double, float, double)
SN_MFMA_INST(double, double, float)
SN_MFMA_INST(double, double, double)
SN_MFMA_INST(double, float, bf16_t)
SN_MFMA_INST(float, float, bf16_t)
SN_MFMA_INST(bf16_t, float, float)
#undef SN_MFMA_INST

}  // namespace sn
