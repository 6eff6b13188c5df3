// Weight gradients for training (paper section 5.1, eq 9): the adjoint of the energy with
// respect to every model weight, seeded per atom with the upstream gradient of its
// structure's energy.
//
// Every weight of a channel-mixing layer, of the radial MLP, of the embedding and of the
// readout enters the energy through a contraction over rows (atoms x m components, or
// undirected edge pairs), so its gradient is a reduction over those rows:
//   dW[k][n] = sum_r A[r][k] B[r][n]
// with A the layer's input rows and B the adjoint of its output rows.  The rows are cut
// into fixed chunks; each chunk's 16 x 16 output tiles are accumulated in float64 by one
// block (rows staged through LDS), and a second kernel adds the chunks in chunk order, so
// the result does not depend on scheduling (no atomics).
#include "kernels.h"

namespace sn {

constexpr int kWgTile = 16;  // output tile edge
constexpr int kWgRows = 64;  // rows staged per LDS round

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_wgrad_partial(int64_t rows, int K, int N,
                                                       const TA* __restrict__ A, RowMap am,
                                                       const int* __restrict__ aidx,
                                                       const int* __restrict__ onehot,
                                                       const TB* __restrict__ B, RowMap bm,
                                                       int64_t chunk, double* __restrict__ partial) {
  __shared__ double sA[kWgRows][kWgTile + 1];
  __shared__ double sB[kWgRows][kWgTile + 1];
  const int tid = threadIdx.x, tn = tid & 15, tk = tid >> 4;
  const int n0 = blockIdx.x * kWgTile, k0 = blockIdx.y * kWgTile;
  const int64_t r0 = (int64_t)blockIdx.z * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double acc = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kWgRows) {
    for (int i = tid; i < kWgRows * kWgTile; i += 256) {
      const int rr = i / kWgTile, cc = i % kWgTile;
      const int64_t r = rb + rr;
      double va = 0.0, vb = 0.0;
      if (r < r1) {
        const int64_t ra = aidx ? (int64_t)aidx[r] : r;
        if (k0 + cc < K)
          va = onehot ? (onehot[ra] == k0 + cc ? 1.0 : 0.0) : (double)sload(A[am(ra) + k0 + cc]);
        if (n0 + cc < N) vb = (double)sload(B[bm(r) + n0 + cc]);
      }
      sA[rr][cc] = va;
      sB[rr][cc] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < kWgRows; ++rr) acc += sA[rr][tk] * sB[rr][tn];
    __syncthreads();
  }
  if (k0 + tk < K && n0 + tn < N)
    partial[((int64_t)blockIdx.z * K + k0 + tk) * N + n0 + tn] = acc;
}

// out[i] = scale * sum over chunks c (in order) of partial[c][i]
__global__ void k_wgrad_reduce(int nchunk, int64_t kn, const double* __restrict__ partial,
                               double scale, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kn) return;
  double v = 0.0;
  for (int c = 0; c < nchunk; ++c) v += partial[(int64_t)c * kn + i];
  out[i] = scale * v;
}

int64_t wgrad_chunks(int64_t rows) {
  // about 4,096 rows per chunk, at most 256 chunks
  int64_t c = (rows + 4095) / 4096;
  return c < 1 ? 1 : (c > 256 ? 256 : c);
}

template <typename TA, typename TB>
void launch_wgrad(int64_t rows, int K, int N, const TA* A, RowMap am, const int* aidx,
                  const int* onehot, const TB* B, RowMap bm, double scale, double* partial,
                  double* out, hipStream_t s) {
  const int64_t nchunk = wgrad_chunks(rows);
  const int64_t chunk = rows > 0 ? (rows + nchunk - 1) / nchunk : 1;
  if (rows > 0) {
    dim3 grid((unsigned)((N + kWgTile - 1) / kWgTile), (unsigned)((K + kWgTile - 1) / kWgTile),
              (unsigned)nchunk);
    k_wgrad_partial<TA, TB><<<grid, 256, 0, s>>>(rows, K, N, A, am, aidx, onehot, B, bm, chunk,
                                                partial);
  } else {
    // no rows: the gradient is zero
    const int64_t kn = (int64_t)K * N;
    k_wgrad_reduce<<<(unsigned)((kn + 255) / 256), 256, 0, s>>>(0, kn, partial, scale, out);
    return;
  }
  const int64_t kn = (int64_t)K * N;
  k_wgrad_reduce<<<(unsigned)((kn + 255) / 256), 256, 0, s>>>((int)nchunk, kn, partial, scale, out);
}

// per local row: the upstream gradient of its structure's energy (region r of structure b is
// b * regions_per_struct + subdomain)
__global__ void k_atom_grad(int n, const int* __restrict__ region, int regions_per_struct,
                            const double* __restrict__ grad, double* __restrict__ g_atom) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g_atom[i] = grad[region[i] / regions_per_struct];
}

// dE/dh of the last block's outputs, seeded per row: sigma g_i v (v = Wr1 Wr2), zero beyond C0
template <typename H>
__global__ void k_seed_rows(int n, const double* __restrict__ v, int C0, double sigma,
                            const double* __restrict__ g_atom, H* __restrict__ dh, int ldh) {
  const int r = blockIdx.x;
  const double g = sigma * g_atom[r];
  for (int k = threadIdx.x; k < ldh; k += blockDim.x)
    dh[(int64_t)r * ldh + k] = (H)(k < C0 ? g * v[k] : 0.0);
}

// readout weights from u = sum_i g_i h_i (C0): E_i = sigma (h_i Wr1) Wr2 + mu, so
//   dWr1[a][b] = sigma u[a] Wr2[b],  dWr2[b] = sigma sum_a Wr1[a][b] u[a]
__global__ void k_readout_wgrad(int C0, const double* __restrict__ u, const double* __restrict__ wr1,
                                const double* __restrict__ wr2, double sigma,
                                double* __restrict__ g_wr1, double* __restrict__ g_wr2) {
  const int H = C0 / 2;
  for (int i = threadIdx.x; i < C0 * H; i += blockDim.x) g_wr1[i] = sigma * u[i / H] * wr2[i % H];
  for (int b = threadIdx.x; b < H; b += blockDim.x) {
    double v = 0.0;
    for (int a = 0; a < C0; ++a) v += wr1[a * H + b] * u[a];
    g_wr2[b] = sigma * v;
  }
}

void launch_atom_grad(int n, const int* region, int regions_per_struct, const double* grad,
                      double* g_atom, hipStream_t s) {
  if (n > 0)
    k_atom_grad<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, region, regions_per_struct, grad, g_atom);
}
template <typename H>
void launch_seed_rows(int n, const double* v, int C0, double sigma, const double* g_atom, H* dh,
                      int ldh, hipStream_t s) {
  if (n > 0) k_seed_rows<H><<<n, 128, 0, s>>>(n, v, C0, sigma, g_atom, dh, ldh);
}
template void launch_seed_rows<double>(int, const double*, int, double, const double*, double*, int,
                                       hipStream_t);
template void launch_seed_rows<float>(int, const double*, int, double, const double*, float*, int,
                                      hipStream_t);
void launch_readout_wgrad(int C0, const double* u, const double* wr1, const double* wr2,
                          double sigma, double* g_wr1, double* g_wr2, hipStream_t s) {
  k_readout_wgrad<<<1, 256, 0, s>>>(C0, u, wr1, wr2, sigma, g_wr1, g_wr2);
}

// positions moved along a direction: out_i = pos_i + eps (v_i + U_b pos_i), b the structure of
// atom i (U row-major 3 x 3 per structure)
__global__ void k_perturb(int64_t n, const double* __restrict__ pos, const double* __restrict__ v,
                          const double* __restrict__ U, const int* __restrict__ atom_struct,
                          double eps, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* u = U + 9 * atom_struct[i];
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  out[3 * i] = x + eps * (v[3 * i] + u[0] * x + u[1] * y + u[2] * z);
  out[3 * i + 1] = y + eps * (v[3 * i + 1] + u[3] * x + u[4] * y + u[5] * z);
  out[3 * i + 2] = z + eps * (v[3 * i + 2] + u[6] * x + u[7] * y + u[8] * z);
}

// y += a x (float64)
__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void k_fill_f64(int64_t n, double v, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

void launch_perturb(int64_t n, const double* pos, const double* v, const double* U,
                    const int* atom_struct, double eps, double* out, hipStream_t s) {
  if (n > 0)
    k_perturb<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, pos, v, U, atom_struct, eps, out);
}
void launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n > 0) k_axpy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, a, x, y);
}
void launch_fill_f64(int64_t n, double v, double* y, hipStream_t s) {
  if (n > 0) k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, v, y);
}

#define SN_WG_INST(TA, TB)                                                                      \
  template void launch_wgrad<TA, TB>(int64_t, int, int, const TA*, RowMap, const int*,           \
                                     const int*, const TB*, RowMap, double, double*, double*,     \
                                     hipStream_t);
SN_WG_INST(double, double)
SN_WG_INST(float, double)
SN_WG_INST(float, float)
SN_WG_INST(double, float)
SN_WG_INST(bf16_t, float)
#undef SN_WG_INST

}  // namespace sn
