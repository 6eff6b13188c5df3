// Dense contractions: row-mapped GEMM for the channel-mixing linears and the
// last radial-MLP layer, and the two hidden radial-MLP layers.
//
// Channel mixing (Lin1, Linsc, Lin2, paper section 5.1 and Fig 2b) acts on
// each degree block independently and identically for every m, so with the
// channel index innermost each (atom, m) pair is one GEMM row; RowMap
// addresses those rows inside the interleaved feature rows.
#include "kernels.h"

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

template <typename T, int NB, int H>
__global__ __launch_bounds__(256) void k_mlp_bwd(int64_t E, const int* __restrict__ rows,
                                                  const T* __restrict__ rho,
                                                  const T* __restrict__ Wa, const T* __restrict__ Wb,
                                                  T c, const T* __restrict__ dz2,
                                                  T* __restrict__ drho, int accumulate) {
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
  }
  for (int j2 = 0; j2 < H; ++j2) {
    T a = T(0);
#pragma unroll
    for (int j = 0; j < H; ++j) a += z1[j] * sWb[j * H + j2];
    T da = dz2[e * H + j2] * act_grad(a, c);
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
                           hipStream_t s) {
  if (E <= 0) return;
  k_mlp_bwd<T, 8, 64><<<(unsigned)((E + 255) / 256), 256, 0, s>>>(E, rows, rho, Wa, Wb, c, dz2,
                                                                  drho, accumulate ? 1 : 0);
}

template <typename T>
__global__ void k_pair_sum(int64_t np, const int* __restrict__ pe1, const int* __restrict__ pe2,
                           const T* __restrict__ dw, int P, T* __restrict__ out) {
  // dE/dw is pair-major: rows 2p and 2p + 1 hold the pair's two directions
  const int64_t p = blockIdx.x;
  const int64_t a = 2 * p * P;
  const int b = pe2[p];
  for (int k = threadIdx.x; k < P; k += blockDim.x)
    out[p * P + k] = dw[a + k] + (b >= 0 ? dw[a + P + k] : T(0));
}

template <typename T>
void launch_pair_sum(int64_t np, const int* pe1, const int* pe2, const T* dw, int P, T* out,
                     hipStream_t s) {
  if (np > 0) k_pair_sum<T><<<(unsigned)np, 128, 0, s>>>(np, pe1, pe2, dw, P, out);
}

#define SN_MLPV_INST(T)                                                                          \
  template void launch_mlp_hidden_fwd<T>(int64_t, const int*, const T*, int, int, const T*,      \
                                         const T*, T, T*, hipStream_t);                          \
  template void launch_mlp_hidden_bwd<T>(int64_t, const int*, const T*, int, int, const T*,      \
                                         const T*, T, const T*, T*, bool, hipStream_t);          \
  template void launch_pair_sum<T>(int64_t, const int*, const int*, const T*, int, T*, hipStream_t);
SN_MLPV_INST(float)
SN_MLPV_INST(double)
#undef SN_MLPV_INST

}  // namespace sn
