// Dense contractions: row-mapped GEMM for the channel-mixing linears and the
// last radial-MLP layer, and the two hidden radial-MLP layers.
//
// Channel mixing (Lin1, Linsc, Lin2, paper section 5.1 and Fig 2b) acts on
// each degree block independently and identically for every m, so with the
// channel index innermost each (atom, m) pair is one GEMM row; RowMap
// addresses those rows inside the interleaved feature rows.
#include "kernels.h"

#include <type_traits>

namespace sn {

// ------------------------------------------------------------------ generic tiled GEMM
constexpr int GT = 64;   // tile rows / cols
constexpr int GK = 32;   // k step

template <typename TACC, typename T>
__device__ inline TACC load_operand(T v, bool bf16) {
  if (bf16) return (TACC)__bfloat162float(__float2bfloat16((float)v));
  return (TACC)v;
}

// C[M x N] (=|+=) alpha * A[M x K] op(B), with operand types TA/TB, result type TC
// and accumulation in TACC.  64 x 64 tile per 256-thread block, 4 x 4 per thread.
template <typename TACC>
struct ValuLds {
  TACC a[GK][GT + 4];
  TACC b[GK][GT + 4];
};

// one 64 x 64 output tile (rows m0.., columns n0..)
template <typename TA, typename TB, typename TC, typename TACC, bool BT>
__device__ inline void gemm_valu_tile(int64_t M, int N, int K, const TA* __restrict__ A, RowMap am,
                                      const TB* __restrict__ B, int ldb, TC* __restrict__ C,
                                      RowMap cm, TACC alpha, int accumulate, int bf16, int64_t m0,
                                      int n0, ValuLds<TACC>& L) {
  auto& As = L.a;
  auto& Bs = L.b;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  TACC acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = TACC(0);
  // A: 8 consecutive k of row ar; B: k-rows bk and bk + 16, 4 consecutive n.  The next
  // k-slab is loaded into registers while the current one is multiplied; every load is
  // issued from a clamped address and masked afterwards (no load under a branch).
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  const int64_t agm = m0 + ar;
  const bool a_ok = agm < M;
  const int64_t arow = a_ok ? am(agm) : 0;
  const int bk = tid >> 4, bn = (tid & 15) * 4;
  TACC ra[8], rb[2][4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + ak + j;
      const TACC v = load_operand<TACC>(A[arow + min(k, K - 1)], bf16);
      ra[j] = (a_ok && k < K) ? v : TACC(0);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + bn + j, k = k0 + bk + 16 * h;
        const int nc = min(n, N - 1), kc = min(k, K - 1);
        const TACC v =
            load_operand<TACC>(BT ? B[(int64_t)nc * ldb + kc] : B[(int64_t)kc * ldb + nc], bf16);
        rb[h][j] = (k < K && n < N) ? v : TACC(0);
      }
  };
  if (K > 0) fetch(0);  // (K = 0: no loads; the tile is written as zeros)
  for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
    for (int j = 0; j < 8; ++j) As[ak + j][ar] = ra[j];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[bk + 16 * h][bn + j] = rb[h][j];
    __syncthreads();
    if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      TACC a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int64_t row = m0 + ty * 4 + i;
    if (row >= M) continue;
    TC* c = C + cm(row);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int col = n0 + tx * 4 + j;
      if (col >= N) continue;
      TACC v = alpha * acc[i][j];
      c[col] = accumulate ? (TC)((TACC)c[col] + v) : (TC)v;
    }
  }
}

// ------------------------------------------------------------------ float64 matrix cores
// The float64-accumulated contractions (the self-connection Linsc of every form; every
// contraction of the FP64 form) on v_mfma_f64_16x16x4_f64: 64 x 64 block tile, four waves
// of 32 x 32 (2 x 2 MFMA tiles of 16 x 16), k-slabs of 16 staged in double-buffered LDS
// with the next slab loaded into registers while the current one is multiplied.  Operand
// layout (lane l): A[row l%16][k l/16], B[k l/16][col l%16]; result register r of lane l
// holds row l/16 + 4 r of column l%16 (rows interleaved, unlike the float32 16x16x4 form).
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int DK = 16;
struct F64Lds {
  double a[2][64][DK + 1];
  double b[2][64][DK + 1];  // stored [n][k]
};

template <typename TA, typename TB, typename TC, bool BT>
__device__ inline void gemm_f64_tile(int64_t M, int N, int K, const TA* __restrict__ A, RowMap am,
                                     const TB* __restrict__ B, int ldb, TC* __restrict__ C,
                                     RowMap cm, double alpha, int accumulate, int64_t m0, int n0,
                                     F64Lds& L) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  doublex4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  // A: row tid/4, k = 4 (tid%4) .. +3; B: 64 x 16 values, 4 per thread (n tid/4, k 4 (tid%4)
  // .. +3 when B is [n][k]; k tid/16, n 4 (tid%16) .. +3 when B is [k][n]).  Loads come from
  // clamped addresses and are masked afterwards.
  const int ar = tid >> 2, ak = (tid & 3) * 4;
  const bool a_ok = m0 + ar < M;
  const int64_t arow = a_ok ? am(m0 + ar) : 0;
  const int bn = BT ? tid >> 2 : (tid & 15) * 4;
  const int bk = BT ? (tid & 3) * 4 : tid >> 4;
  double ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + ak + e;
      const double v = (double)A[arow + min(k, K - 1)];
      ra[e] = (a_ok && k < K) ? v : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int n = n0 + bn + (BT ? 0 : e), k = k0 + bk + (BT ? e : 0);
      const int nc = min(n, N - 1), kc = min(k, K - 1);
      const double v = (double)(BT ? B[(int64_t)nc * ldb + kc] : B[(int64_t)kc * ldb + nc]);
      rb[e] = (n < N && k < K) ? v : 0.0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) L.a[buf][ar][ak + e] = ra[e];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (BT) L.b[buf][bn][bk + e] = rb[e];
      else L.b[buf][bn + e][bk] = rb[e];
    }
  };
  if (K > 0) fetch(0);
  int buf = 0;
  const int r = lane & 15, kq = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += DK) {
    stage(buf);
    __syncthreads();
    if (k0 + DK < K) fetch(k0 + DK);
#pragma unroll
    for (int kk = 0; kk < DK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = L.a[buf][wr + i * 16 + r][kk + kq];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = L.b[buf][wc + j * 16 + r][kk + kq];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    buf ^= 1;
  }
  const int row_q = lane >> 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc + j * 16 + r;
      if (col >= N) continue;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t row = m0 + wr + i * 16 + row_q + 4 * rr;
        if (row >= M) continue;
        TC* c = C + cm(row) + col;
        const double v = alpha * acc[i][j][rr];
        *c = accumulate ? (TC)((double)*c + v) : (TC)v;
      }
    }
}

template <typename TA, typename TB, typename TC, bool BT>
__global__ __launch_bounds__(256) void k_gemm_f64(int64_t M, int N, int K, const TA* __restrict__ A,
                                                   RowMap am, const TB* __restrict__ B, int ldb,
                                                   TC* __restrict__ C, RowMap cm, double alpha,
                                                   int accumulate, int nbn, int64_t ntiles,
                                                   int64_t chunk) {
  __shared__ F64Lds lds;
  const int64_t p = blockIdx.x;
  const int64_t tile = (p % 8) * chunk + p / 8;  // XCD-contiguous tile order
  if (tile >= ntiles) return;
  gemm_f64_tile<TA, TB, TC, BT>(M, N, K, A, am, B, ldb, C, cm, alpha, accumulate,
                                (tile / nbn) * 64, (int)(tile % nbn) * 64, lds);
}

template <typename TA, typename TB, typename TC, typename TACC, bool BT>
__global__ __launch_bounds__(256) void k_gemm_valu(int64_t M, int N, int K, const TA* __restrict__ A,
                                                    RowMap am, const TB* __restrict__ B, int ldb,
                                                    TC* __restrict__ C, RowMap cm, TACC alpha,
                                                    int accumulate, int bf16) {
  __shared__ ValuLds<TACC> lds;
  gemm_valu_tile<TA, TB, TC, TACC, BT>(M, N, K, A, am, B, ldb, C, cm, alpha, accumulate, bf16,
                                       (int64_t)blockIdx.x * GT, blockIdx.y * GT, lds);
}

// grouped launch: problem q owns blocks [tile0[q], tile0[q + 1]), nbn[q] column tiles per row
template <typename TA, typename TB, typename TC>
struct ValuGroupArgs {
  GemmDesc<TA, TB, TC> d[kMaxGemmGroup];
  int64_t tile0[kMaxGemmGroup + 1];
  int nbn[kMaxGemmGroup];
  int n;
};

template <typename TA, typename TB, typename TC, bool BT>
__global__ __launch_bounds__(256) void k_gemm_f64_g(ValuGroupArgs<TA, TB, TC> g) {
  __shared__ F64Lds lds;
  const int64_t tile = blockIdx.x;
  int q = 0;
  while (q + 1 < g.n && tile >= g.tile0[q + 1]) ++q;
  const GemmDesc<TA, TB, TC>& d = g.d[q];
  const int64_t t = tile - g.tile0[q];
  gemm_f64_tile<TA, TB, TC, BT>(d.M, d.N, d.K, d.A, d.am, d.B, d.ldb, d.C, d.cm, d.alpha,
                                d.accumulate, (t / g.nbn[q]) * GT, (int)(t % g.nbn[q]) * GT, lds);
}

template <typename TA, typename TB, typename TC, typename TACC, bool BT>
__global__ __launch_bounds__(256) void k_gemm_valu_g(ValuGroupArgs<TA, TB, TC> g, int bf16) {
  __shared__ ValuLds<TACC> lds;
  const int64_t tile = blockIdx.x;
  int q = 0;
  while (q + 1 < g.n && tile >= g.tile0[q + 1]) ++q;
  const GemmDesc<TA, TB, TC>& d = g.d[q];
  const int64_t t = tile - g.tile0[q];
  gemm_valu_tile<TA, TB, TC, TACC, BT>(d.M, d.N, d.K, d.A, d.am, d.B, d.ldb, d.C, d.cm,
                                       (TACC)d.alpha, d.accumulate, bf16, (t / g.nbn[q]) * GT,
                                       (int)(t % g.nbn[q]) * GT, lds);
}

template <typename TA, typename TB, typename TC, typename TACC>
void launch_gemm(int64_t M, int N, int K, const TA* A, RowMap am, const TB* B, int ldb, bool bt,
                 TC* C, RowMap cm, TACC alpha, bool accumulate, bool bf16_operands, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  if (std::is_same<TACC, double>::value && !bf16_operands) {  // float64 matrix cores
    const int nbn = (N + 63) / 64;
    const int64_t ntiles = ((M + 63) / 64) * nbn;
    const int64_t chunk = (ntiles + 7) / 8;
    const unsigned g = (unsigned)(chunk * 8);
    if (bt)
      k_gemm_f64<TA, TB, TC, true><<<g, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm, (double)alpha,
                                                     accumulate ? 1 : 0, nbn, ntiles, chunk);
    else
      k_gemm_f64<TA, TB, TC, false><<<g, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm, (double)alpha,
                                                      accumulate ? 1 : 0, nbn, ntiles, chunk);
    return;
  }
  dim3 grid((unsigned)((M + GT - 1) / GT), (unsigned)((N + GT - 1) / GT));
  if (bt)
    k_gemm_valu<TA, TB, TC, TACC, true><<<grid, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm, alpha,
                                                             accumulate, bf16_operands);
  else
    k_gemm_valu<TA, TB, TC, TACC, false><<<grid, 256, 0, s>>>(M, N, K, A, am, B, ldb, C, cm, alpha,
                                                              accumulate, bf16_operands);
}

template <typename TA, typename TB, typename TC, typename TACC>
void launch_gemm_group(int n, const GemmDesc<TA, TB, TC>* d, bool bt, bool bf16_operands,
                       hipStream_t s) {
  ValuGroupArgs<TA, TB, TC> g{};
  for (int q = 0; q < n && q < kMaxGemmGroup; ++q)
    if (d[q].M > 0 && d[q].N > 0) g.d[g.n++] = d[q];
  int64_t tiles = 0;
  for (int q = 0; q < g.n; ++q)
    tiles += ((g.d[q].M + GT - 1) / GT) * ((g.d[q].N + GT - 1) / GT);
  if (n > kMaxGemmGroup || g.n <= 1 || tiles > kGroupMaxTiles) {  // one launch per problem
    for (int q = 0; q < n; ++q)
      launch_gemm<TA, TB, TC, TACC>(d[q].M, d[q].N, d[q].K, d[q].A, d[q].am, d[q].B, d[q].ldb, bt,
                                    d[q].C, d[q].cm, (TACC)d[q].alpha, d[q].accumulate != 0,
                                    bf16_operands, s);
    return;
  }
  g.tile0[0] = 0;
  for (int q = 0; q < g.n; ++q) {
    g.nbn[q] = (g.d[q].N + GT - 1) / GT;
    g.tile0[q + 1] = g.tile0[q] + ((g.d[q].M + GT - 1) / GT) * g.nbn[q];
  }
  const unsigned grid = (unsigned)g.tile0[g.n];
  if (std::is_same<TACC, double>::value && !bf16_operands) {
    if (bt) k_gemm_f64_g<TA, TB, TC, true><<<grid, 256, 0, s>>>(g);
    else k_gemm_f64_g<TA, TB, TC, false><<<grid, 256, 0, s>>>(g);
    return;
  }
  if (bt)
    k_gemm_valu_g<TA, TB, TC, TACC, true><<<grid, 256, 0, s>>>(g, bf16_operands ? 1 : 0);
  else
    k_gemm_valu_g<TA, TB, TC, TACC, false><<<grid, 256, 0, s>>>(g, bf16_operands ? 1 : 0);
}

#define SN_GEMM_INST(TA, TB, TC, TACC)                                                          \
  template void launch_gemm<TA, TB, TC, TACC>(int64_t, int, int, const TA*, RowMap, const TB*,   \
                                              int, bool, TC*, RowMap, TACC, bool, bool,          \
                                              hipStream_t);                                      \
  template void launch_gemm_group<TA, TB, TC, TACC>(int, const GemmDesc<TA, TB, TC>*, bool, bool, \
                                                    hipStream_t);
SN_GEMM_INST(double, double, double, double)
SN_GEMM_INST(double, double, float, double)
SN_GEMM_INST(float, float, double, float)
SN_GEMM_INST(double, float, float, float)
SN_GEMM_INST(double, float, double, float)
SN_GEMM_INST(float, float, float, float)
#undef SN_GEMM_INST

// ------------------------------------------------------------------ radial MLP hidden layers
// z2 = phi(phi(rho Wa) Wb); phi(z) = c z sigmoid(z); no biases.  One thread per edge,
// weights in LDS (read as broadcasts).
template <typename T, int NB, int H>
__global__ __launch_bounds__(256) void k_mlp_fwd(int64_t E, const int* __restrict__ rows,
                                                  const T* __restrict__ rho,
                                                  const T* __restrict__ Wa, const T* __restrict__ Wb,
                                                  T c, T* __restrict__ z2) {
  __shared__ T sWa[NB * H];
  __shared__ T sWb[H * H];
  for (int i = threadIdx.x; i < NB * H; i += blockDim.x) sWa[i] = Wa[i];
  for (int i = threadIdx.x; i < H * H; i += blockDim.x) sWb[i] = Wb[i];
  __syncthreads();
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  T r[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) r[k] = rho[(int64_t)rows[e] * NB + k];
  T z1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) a += r[k] * sWa[k * H + j];
    z1[j] = act(a, c);
  }
  for (int j2 = 0; j2 < H; ++j2) {
    T a = T(0);
#pragma unroll
    for (int j = 0; j < H; ++j) a += z1[j] * sWb[j * H + j2];
    z2[e * H + j2] = act(a, c);
  }
}

// With z1o, da1o, da2o (training): also the per-pair hidden activation z1 = phi(a1) and the
// pre-activation gradients da1 = dE/da1, da2 = dE/da2 that the weight gradients need.
template <typename T, int NB, int H>
__global__ __launch_bounds__(256) void k_mlp_bwd(int64_t E, const int* __restrict__ rows,
                                                  const T* __restrict__ rho,
                                                  const T* __restrict__ Wa, const T* __restrict__ Wb,
                                                  T c, const T* __restrict__ dz2,
                                                  T* __restrict__ drho, int accumulate,
                                                  T* __restrict__ z1o, T* __restrict__ da1o,
                                                  T* __restrict__ da2o) {
  __shared__ T sWa[NB * H];
  __shared__ T sWb[H * H];
  for (int i = threadIdx.x; i < NB * H; i += blockDim.x) sWa[i] = Wa[i];
  for (int i = threadIdx.x; i < H * H; i += blockDim.x) sWb[i] = Wb[i];
  __syncthreads();
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  T r[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) r[k] = rho[(int64_t)rows[e] * NB + k];
  T z1[H], dz1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) a += r[k] * sWa[k * H + j];
    z1[j] = act(a, c);
    dz1[j] = T(0);
    if (z1o) z1o[e * H + j] = z1[j];
  }
  for (int j2 = 0; j2 < H; ++j2) {
    T a = T(0);
#pragma unroll
    for (int j = 0; j < H; ++j) a += z1[j] * sWb[j * H + j2];
    T da = dz2[e * H + j2] * act_grad(a, c);
    if (da2o) da2o[e * H + j2] = da;
#pragma unroll
    for (int j = 0; j < H; ++j) dz1[j] += da * sWb[j * H + j2];
  }
  T dr[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) dr[k] = T(0);
#pragma unroll
  for (int j = 0; j < H; ++j) {
    T a = T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) a += r[k] * sWa[k * H + j];
    T da = dz1[j] * act_grad(a, c);
    if (da1o) da1o[e * H + j] = da;
#pragma unroll
    for (int k = 0; k < NB; ++k) dr[k] += da * sWa[k * H + j];
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int64_t o = (int64_t)rows[e] * NB + k;
    drho[o] = accumulate ? drho[o] + dr[k] : dr[k];
  }
}

template <typename T>
void launch_mlp_hidden_fwd(int64_t E, const int* rows, const T* rho, int nb, int hidden,
                           const T* Wa, const T* Wb, T c, T* z2, hipStream_t s) {
  if (E <= 0) return;
  // nb == 8, hidden == 64 (checked at model load)
  k_mlp_fwd<T, 8, 64><<<(unsigned)((E + 255) / 256), 256, 0, s>>>(E, rows, rho, Wa, Wb, c, z2);
}
template <typename T>
void launch_mlp_hidden_bwd(int64_t E, const int* rows, const T* rho, int nb, int hidden,
                           const T* Wa, const T* Wb, T c, const T* dz2, T* drho, bool accumulate,
                           hipStream_t s, T* z1, T* da1, T* da2) {
  if (E <= 0) return;
  k_mlp_bwd<T, 8, 64><<<(unsigned)((E + 255) / 256), 256, 0, s>>>(
      E, rows, rho, Wa, Wb, c, dz2, drho, accumulate ? 1 : 0, z1, da1, da2);
}

template <typename S, typename T>
__global__ void k_pair_sum(int64_t np, const int* __restrict__ pe1, const int* __restrict__ pe2,
                           const S* __restrict__ dw, int P, T* __restrict__ out) {
  // dE/dw is pair-major: rows 2p and 2p + 1 hold the pair's two directions
  const int64_t p = blockIdx.x;
  const int64_t a = 2 * p * P;
  const int b = pe2[p];
  for (int k = threadIdx.x; k < P; k += blockDim.x)
    out[p * P + k] = T(sload(dw[a + k])) + (b >= 0 ? T(sload(dw[a + P + k])) : T(0));
}

template <typename S, typename T>
void launch_pair_sum(int64_t np, const int* pe1, const int* pe2, const S* dw, int P, T* out,
                     hipStream_t s) {
  if (np > 0) k_pair_sum<S, T><<<(unsigned)np, 128, 0, s>>>(np, pe1, pe2, dw, P, out);
}

#define SN_MLPV_INST(T)                                                                          \
  template void launch_mlp_hidden_fwd<T>(int64_t, const int*, const T*, int, int, const T*,      \
                                         const T*, T, T*, hipStream_t);                          \
  template void launch_mlp_hidden_bwd<T>(int64_t, const int*, const T*, int, int, const T*,      \
                                         const T*, T, const T*, T*, bool, hipStream_t, T*, T*,   \
                                         T*);                                                    \
  template void launch_pair_sum<T, T>(int64_t, const int*, const int*, const T*, int, T*,        \
                                      hipStream_t);
SN_MLPV_INST(float)
SN_MLPV_INST(double)
#undef SN_MLPV_INST
template void launch_pair_sum<bf16_t, float>(int64_t, const int*, const int*, const bf16_t*, int,
                                             float*, hipStream_t);

}  // namespace sn
