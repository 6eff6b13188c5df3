// Node-level kernels and deterministic reductions.
//
//  * embedding (h^(1) = W_emb[species], section 2 and section 3.1: a ghost's
//    first features come from its own species, so block 1 needs no refresh);
//  * ghost refresh: ghost rows copy their owner's rows before every block
//    after the first (forward communication, section 3.1, Fig 3d);
//  * gate nonlinearity (forward and adjoint);
//  * readout E_i = sigma (h_i Wr1) Wr2 + mu_s (eq 1 with the shift/scale of
//    section 5.1); Wr1 Wr2 is a single C0-vector because no activation sits
//    between the two linears;
//  * sender-side segmented sums of per-edge gradient rows and the ghost fold
//    (reverse communication of dE/dh and of partial forces, Fig 3e-f);
//  * atomic forces from edge gradients (eq 6), virial and energy in float64.
// Every reduction has a fixed order: no floating-point atomics.
#include "kernels.h"

namespace sn {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


template <typename T>
__global__ void k_embed(int rows, const int* __restrict__ spec, const T* __restrict__ Wemb, int C0,
                        T* __restrict__ h, int ldh) {
  int r = blockIdx.x;
  const T* src = Wemb + (int64_t)spec[r] * C0;
  for (int c = threadIdx.x; c < C0; c += blockDim.x) h[(int64_t)r * ldh + c] = src[c];
}

template <typename T>
__global__ void k_ghost_refresh(int n_local, const int* __restrict__ owner, T* __restrict__ x,
                                int width) {
  int g = blockIdx.x;
  const T* src = x + (int64_t)owner[g] * width;
  T* dst = x + (int64_t)(n_local + g) * width;
  for (int c = threadIdx.x; c < width; c += blockDim.x) dst[c] = src[c];
}

// y: gate-input row (l0: C0 scalars then gates for each l > 0 channel; l > 0 blocks)
// h: output row (l0: C0; l > 0 blocks).  Last block: h0 = phi(y0) over C0 entries.
template <typename T>
__global__ void k_gate_fwd(int n, int last, IrrepLayout yl, IrrepLayout hl, const T* __restrict__ y,
                           T* __restrict__ h, T c) {
  int r = blockIdx.x;
  const T* yr = y + (int64_t)r * yl.width;
  T* hr = h + (int64_t)r * hl.width;
  const int C0 = hl.mul[0];
  for (int k = threadIdx.x; k < C0; k += blockDim.x) hr[hl.off[0] + k] = act(yr[yl.off[0] + k], c);
  if (last) return;
  int goff = C0;
  for (int l = 1; l < kNumL; ++l) {
    const int mul = hl.mul[l];
    if (mul == 0) continue;
    const int nm = 2 * l + 1;
    for (int k = threadIdx.x; k < nm * mul; k += blockDim.x) {
      const int u = k % mul;
      const T gv = act(yr[yl.off[0] + goff + u], c);
      hr[hl.off[l] + k] = gv * yr[yl.off[l] + k];
    }
    goff += mul;
  }
}

// y (the gate input) in the forward node type TY, gradients in TG; arithmetic in TY
template <typename TY, typename TG>
__global__ void k_gate_bwd(int n, int last, IrrepLayout yl, IrrepLayout hl, const TY* __restrict__ y,
                           const TG* __restrict__ dh, TG* __restrict__ dy, TY c) {
  int r = blockIdx.x;
  const TY* yr = y + (int64_t)r * yl.width;
  const TG* dhr = dh + (int64_t)r * hl.width;
  TG* dyr = dy + (int64_t)r * yl.width;
  const int C0 = hl.mul[0];
  for (int k = threadIdx.x; k < C0; k += blockDim.x)
    dyr[yl.off[0] + k] = (TG)((TY)dhr[hl.off[0] + k] * act_grad(yr[yl.off[0] + k], c));
  if (last) return;
  int goff = C0;
  for (int l = 1; l < kNumL; ++l) {
    const int mul = hl.mul[l];
    if (mul == 0) continue;
    const int nm = 2 * l + 1;
    for (int k = threadIdx.x; k < nm * mul; k += blockDim.x) {
      const int u = k % mul;
      dyr[yl.off[l] + k] = (TG)((TY)dhr[hl.off[l] + k] * act(yr[yl.off[0] + goff + u], c));
    }
    for (int u = threadIdx.x; u < mul; u += blockDim.x) {
      TY s = TY(0);
      for (int m = 0; m < nm; ++m)
        s += (TY)dhr[hl.off[l] + m * mul + u] * yr[yl.off[l] + m * mul + u];
      const TY z = yr[yl.off[0] + goff + u];
      dyr[yl.off[0] + goff + u] = (TG)(s * act_grad(z, c));
    }
    goff += mul;
  }
}

template <typename T>
__global__ void k_readout(int n, const T* __restrict__ h, int ldh, const double* __restrict__ v,
                          int C0, double sigma, const double* __restrict__ shift,
                          const int* __restrict__ spec, double* __restrict__ atom_e) {
  // one wave per atom
  int r = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = threadIdx.x % kWave;
  if (r >= n) return;
  double s = 0.0;
  for (int k = lane; k < C0; k += kWave) s += (double)h[(int64_t)r * ldh + k] * v[k];
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) atom_e[r] = sigma * s + shift[spec[r]];
}

template <typename T>
__global__ void k_fill_rows(int n, const double* __restrict__ v, int C0, double scale,
                            T* __restrict__ dh, int ldh) {
  int r = blockIdx.x;
  for (int k = threadIdx.x; k < ldh; k += blockDim.x)
    dh[(int64_t)r * ldh + k] = k < C0 ? T(scale * v[k]) : T(0);
}

// One row per block; each thread owns 4 consecutive columns (one 16-byte load per edge
// in float32) and accumulates in the output type H (float64, or float32 in the bfloat16
// form).  The edge loop is unrolled for memory-level parallelism; the summation order
// stays the sender segment's order.
template <typename T, typename H>
__global__ void k_sender_reduce(int n_rows, const int* __restrict__ sptr, const int* __restrict__ sidx,
                                const T* __restrict__ dxe, int width, H* __restrict__ dx) {
  const int s = blockIdx.x;
  const int a = sptr[s], b = sptr[s + 1];
  for (int c = threadIdx.x * 4; c < width; c += blockDim.x * 4) {
    H acc[4] = {H(0), H(0), H(0), H(0)};
    int q = a;
    for (; q + 4 <= b; q += 4) {
      T v[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T* row = dxe + (int64_t)sidx[q + k] * width + c;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[k][j] = row[j];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] += (H)sload(v[k][j]);
    }
    for (; q < b; ++q) {
      const T* row = dxe + (int64_t)sidx[q] * width + c;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += (H)sload(row[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) dx[(int64_t)s * width + c + j] = acc[j];
  }
}

// dx[o] = dx_ext[o] + sum of the owner's ghost rows dx_ext[n_local + g]
template <typename T>
__global__ void k_ghost_fold(int n_local, const int* __restrict__ gptr, const T* __restrict__ dx_ext,
                             T* __restrict__ dx, int width) {
  int o = blockIdx.x;
  int a = gptr[o], b = gptr[o + 1];
  for (int c = threadIdx.x; c < width; c += blockDim.x) {
    T acc = dx_ext[(int64_t)o * width + c];
    for (int q = a; q < b; ++q) acc += dx_ext[(int64_t)(n_local + q) * width + c];
    dx[(int64_t)o * width + c] = acc;
  }
}

template <typename T>
__global__ void k_dY_reduce(int64_t E, int n_tasks, int NY, const T* __restrict__ part,
                            T* __restrict__ dY, int accumulate) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * NY) return;
  int64_t e = idx / NY;
  int q = (int)(idx % NY);
  T s = T(0);
  for (int t = 0; t < n_tasks; ++t) s += part[(e * n_tasks + t) * NY + q];
  dY[idx] = accumulate ? dY[idx] + s : s;
}

// F_k = sum_{e: recv=k} g_e - sum_{e: send=k} g_e - sum_{ghosts of k} sum_{e: send=ghost} g_e
// F_k = sum of g over k's receiver edges - sum over the edges k and its ghost images send;
// one wave per atom, lanes over the edge lists, combined by a fixed butterfly
__global__ __launch_bounds__(256) void k_forces(int n_local, const int* __restrict__ row_ptr,
                                                const int* __restrict__ sptr,
                                                const int* __restrict__ sidx,
                                                const int* __restrict__ gptr,
                                                const double* __restrict__ g,
                                                double* __restrict__ F) {
  const int k = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (k >= n_local) return;
  const int lane = threadIdx.x & 63;
  double f[3] = {0, 0, 0};
  for (int e = row_ptr[k] + lane; e < row_ptr[k + 1]; e += 64)
    for (int a = 0; a < 3; ++a) f[a] += g[3 * (int64_t)e + a];
  for (int q = sptr[k] + lane; q < sptr[k + 1]; q += 64) {
    const int64_t e = sidx[q];
    for (int a = 0; a < 3; ++a) f[a] -= g[3 * e + a];
  }
  for (int gh = gptr[k]; gh < gptr[k + 1]; ++gh) {
    const int s = n_local + gh;
    for (int q = sptr[s] + lane; q < sptr[s + 1]; q += 64) {
      const int64_t e = sidx[q];
      for (int a = 0; a < 3; ++a) f[a] -= g[3 * e + a];
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int a = 0; a < 3; ++a) f[a] += __shfl_xor(f[a], off);
  if (lane == 0)
    for (int a = 0; a < 3; ++a) F[3 * (int64_t)k + a] = f[a];
}

constexpr int kRedThreads = 256;

// Per-structure segmented sums in fixed order: one block per chunk (structure, begin,
// end) reduces its items with a tree in shared memory; k_seg_finalize adds the chunks of
// every structure in chunk order.
__global__ void k_seg_energy(const int* __restrict__ chunks, const double* __restrict__ atom_e,
                             double* __restrict__ partial) {
  __shared__ double s[kRedThreads];
  const int a = chunks[3 * blockIdx.x + 1], b = chunks[3 * blockIdx.x + 2];
  double v = 0;
  for (int i = a + threadIdx.x; i < b; i += blockDim.x) v += atom_e[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// -d_e (x) g_e summed over the chunk's edges (row-major 3x3)
__global__ void k_seg_virial(const int* __restrict__ chunks, const int* __restrict__ recv,
                             const int* __restrict__ src, const double* __restrict__ pos_ext,
                             const double* __restrict__ g, double* __restrict__ partial) {
  __shared__ double s[kRedThreads][9];
  const int a = chunks[3 * blockIdx.x + 1], b = chunks[3 * blockIdx.x + 2];
  double w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t e = a + threadIdx.x; e < b; e += blockDim.x) {
    int i = recv[e], j = src[e];
    double d[3];
    for (int q = 0; q < 3; ++q) d[q] = pos_ext[3 * j + q] - pos_ext[3 * i + q];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) w[p * 3 + q] -= d[p] * g[3 * e + q];
  }
  for (int q = 0; q < 9; ++q) s[threadIdx.x][q] = w[q];
  __syncthreads();
  for (int off = kRedThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off)
      for (int q = 0; q < 9; ++q) s[threadIdx.x][q] += s[threadIdx.x + off][q];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 9; ++q) partial[blockIdx.x * 9 + q] = s[0][q];
}

// gscale (device, one value per structure, or null for 1) multiplies structure b's sums:
// the upstream gradient dL/dE_b of a backward pass
__global__ void k_seg_finalize(int B, const int* __restrict__ first, const double* __restrict__ partial,
                               int width, double* __restrict__ out, const double* __restrict__ gscale) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * width) return;
  int b = idx / width, q = idx % width;
  double v = 0;
  for (int c = first[b]; c < first[b + 1]; ++c) v += partial[c * width + q];
  out[idx] = (gscale ? gscale[b] : 1.0) * v;
}

// rows back to the caller's atom order; with gscale, row o is multiplied by the value of
// its structure, sid_orig[o] / regions_per_struct
__global__ void k_unpermute(int n, const int* __restrict__ order, const double* __restrict__ in_rows,
                            int width, double* __restrict__ out_rows, const double* __restrict__ gscale,
                            const int* __restrict__ sid_orig, int regions_per_struct) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int o = order[k];
  const double scale = gscale ? gscale[sid_orig[o] / regions_per_struct] : 1.0;
  for (int a = 0; a < width; ++a) out_rows[(int64_t)o * width + a] = scale * in_rows[(int64_t)k * width + a];
}

// Positions of a kept graph after the atoms moved: local rows in cell order from the
// caller's positions plus the lattice translation applied when the graph was built
// (wrap_off), ghost rows = owner row + shift . H.
__global__ void k_refresh_positions(int n, const int* __restrict__ order,
                                    const double* __restrict__ pos, const double* __restrict__ wrap_off,
                                    double* __restrict__ pos_ext) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = order[k];
  for (int a = 0; a < 3; ++a) pos_ext[3 * k + a] = pos[3 * o + a] + wrap_off[3 * k + a];
}
__global__ void k_refresh_ghosts(int n, int n_ghost, const int* __restrict__ owner,
                                 const int* __restrict__ shift, const int* __restrict__ sid,
                                 const StructParams* __restrict__ sp, double* __restrict__ pos_ext) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_ghost) return;
  const int o = owner[g];
  const double* H = sp[sid[n + g]].H;
  const int sx = shift[3 * g], sy = shift[3 * g + 1], sz = shift[3 * g + 2];
  for (int a = 0; a < 3; ++a)
    pos_ext[3 * (int64_t)(n + g) + a] = pos_ext[3 * o + a] + sx * H[a] + sy * H[3 + a] + sz * H[6 + a];
}

// wrap_off[k] = wrapped - original position of local row k (a lattice translation)
__global__ void k_wrap_offsets(int n, const int* __restrict__ order, const double* __restrict__ pos,
                               const double* __restrict__ pos_ext, double* __restrict__ wrap_off) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = order[k];
  for (int a = 0; a < 3; ++a) wrap_off[3 * k + a] = pos_ext[3 * k + a] - pos[3 * o + a];
}

// Velocity Verlet halves (harness of the molecular-dynamics workload):
// stage 0: v += dt/2 a, x += dt v;  stage 1: v += dt/2 a, with a = F * inv_mass.
__global__ void k_verlet(int n, double* __restrict__ pos, double* __restrict__ vel,
                         const double* __restrict__ F, const double* __restrict__ inv_mass,
                         double dt, int stage) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int a = 0; a < 3; ++a) {
    double v = vel[3 * i + a] + 0.5 * dt * F[3 * i + a] * inv_mass[i];
    vel[3 * i + a] = v;
    if (stage == 0) pos[3 * i + a] += dt * v;
  }
}

// Nose-Hoover thermostat (one thermostat on all particles), half-step operator of the
// symmetric Trotter splitting of the equations of motion
//   dv/dt = F/m - xi v,  dxi/dt = (2K - g kT) / Q,  deta/dt = xi:
//   xi += dt/4 G(K);  eta += dt/2 xi;  v *= exp(-xi dt/2);  xi += dt/4 G(K exp(-xi dt)),
// G(K) = (2K - g kT) / Q.  K = sum v^2 / (2 inv_mass) is formed from fixed-order block sums.
// The state {xi, eta, scale, K} stays in device memory.
constexpr int kKinBlock = 256;
__global__ void k_kinetic_partial(int n, const double* __restrict__ vel,
                                  const double* __restrict__ inv_mass, double* __restrict__ part) {
  __shared__ double sh[kKinBlock];
  const int i = blockIdx.x * kKinBlock + threadIdx.x;
  double k = 0.0;
  if (i < n)
    k = 0.5 * (vel[3 * i] * vel[3 * i] + vel[3 * i + 1] * vel[3 * i + 1] +
               vel[3 * i + 2] * vel[3 * i + 2]) / inv_mass[i];
  sh[threadIdx.x] = k;
  __syncthreads();
  for (int o = kKinBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_nh_scalars(int nb, const double* __restrict__ part, double dt, double gkT,
                             double Q, double* __restrict__ st) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double K = 0.0;
  for (int b = 0; b < nb; ++b) K += part[b];
  double xi = st[0];
  xi += 0.25 * dt * (2.0 * K - gkT) / Q;
  st[1] += 0.5 * dt * xi;
  const double sc = exp(-0.5 * dt * xi);
  K *= sc * sc;
  xi += 0.25 * dt * (2.0 * K - gkT) / Q;
  st[0] = xi;
  st[2] = sc;
  st[3] = K;
}
__global__ void k_scale_vel(int n, double* __restrict__ vel, const double* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  vel[i] *= st[2];
}

// max over atoms of |pos - ref|^2: block maxima, then one block over those
__global__ void k_disp_partial(int n, const double* __restrict__ pos, const double* __restrict__ ref,
                               double* __restrict__ part) {
  __shared__ double sh[kKinBlock];
  const int i = blockIdx.x * kKinBlock + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    const double dx = pos[3 * i] - ref[3 * i], dy = pos[3 * i + 1] - ref[3 * i + 1],
                 dz = pos[3 * i + 2] - ref[3 * i + 2];
    d = dx * dx + dy * dy + dz * dz;
  }
  sh[threadIdx.x] = d;
  __syncthreads();
  for (int o = kKinBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_max_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kKinBlock];
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += kKinBlock) m = fmax(m, part[b]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = kKinBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------------------ launchers
int md_partials(int n) { return (int)nblk(n, kKinBlock); }
void launch_nh_half(int n, double* vel, const double* inv_mass, double dt, double gkT, double Q,
                    double* state, double* part, hipStream_t s) {
  if (n <= 0) return;
  const int nb = md_partials(n);
  k_kinetic_partial<<<nb, kKinBlock, 0, s>>>(n, vel, inv_mass, part);
  k_nh_scalars<<<1, 64, 0, s>>>(nb, part, dt, gkT, Q, state);
  k_scale_vel<<<nblk(3 * (int64_t)n, 256), 256, 0, s>>>(n, vel, state);
}
void launch_max_disp2(int n, const double* pos, const double* ref, double* part, double* out,
                      hipStream_t s) {
  if (n <= 0) return;
  const int nb = md_partials(n);
  k_disp_partial<<<nb, kKinBlock, 0, s>>>(n, pos, ref, part);
  k_max_final<<<1, kKinBlock, 0, s>>>(nb, part, out);
}
void launch_refresh_positions(int n, int n_ghost, const int* order, const double* pos,
                              const double* wrap_off, const int* owner, const int* shift,
                              const int* sid_ext, const StructParams* sp, double* pos_ext,
                              hipStream_t s) {
  if (n > 0) k_refresh_positions<<<nblk(n, 256), 256, 0, s>>>(n, order, pos, wrap_off, pos_ext);
  if (n_ghost > 0)
    k_refresh_ghosts<<<nblk(n_ghost, 256), 256, 0, s>>>(n, n_ghost, owner, shift, sid_ext, sp, pos_ext);
}
void launch_wrap_offsets(int n, const int* order, const double* pos, const double* pos_ext,
                         double* wrap_off, hipStream_t s) {
  if (n > 0) k_wrap_offsets<<<nblk(n, 256), 256, 0, s>>>(n, order, pos, pos_ext, wrap_off);
}
void launch_verlet(int n, double* pos, double* vel, const double* F, const double* inv_mass,
                   double dt, int stage, hipStream_t s) {
  if (n > 0) k_verlet<<<nblk(n, 256), 256, 0, s>>>(n, pos, vel, F, inv_mass, dt, stage);
}


template <typename T>
void launch_embed(int rows, const int* spec, const T* Wemb, int C0, T* h, int ldh, hipStream_t s) {
  if (rows > 0) k_embed<T><<<rows, 64, 0, s>>>(rows, spec, Wemb, C0, h, ldh);
}
template <typename T>
void launch_ghost_refresh(int n_local, int n_ghost, const int* owner, T* x, int width, hipStream_t s) {
  if (n_ghost > 0) k_ghost_refresh<T><<<n_ghost, 128, 0, s>>>(n_local, owner, x, width);
}
template <typename T>
void launch_gate_fwd(int n, bool last, IrrepLayout yl, IrrepLayout hl, const T* y, T* h, T c,
                     hipStream_t s) {
  if (n > 0) k_gate_fwd<T><<<n, 128, 0, s>>>(n, last ? 1 : 0, yl, hl, y, h, c);
}
template <typename TY, typename TG>
void launch_gate_bwd(int n, bool last, IrrepLayout yl, IrrepLayout hl, const TY* y, const TG* dh,
                     TG* dy, TY c, hipStream_t s) {
  if (n > 0) k_gate_bwd<TY, TG><<<n, 128, 0, s>>>(n, last ? 1 : 0, yl, hl, y, dh, dy, c);
}
template <typename T>
void launch_readout(int n, const T* h, int ldh, const double* v, int C0, double sigma,
                    const double* shift, const int* spec, double* atom_e, hipStream_t s) {
  if (n > 0) k_readout<T><<<nblk(n, 4), 256, 0, s>>>(n, h, ldh, v, C0, sigma, shift, spec, atom_e);
}
template <typename T>
void launch_fill_rows(int n, const double* v, int C0, double scale, T* dh, int ldh, hipStream_t s) {
  if (n > 0) k_fill_rows<T><<<n, 128, 0, s>>>(n, v, C0, scale, dh, ldh);
}
template <typename T, typename H>
void launch_sender_reduce(int n_rows, const int* sptr, const int* sidx, const T* dxe, int width,
                          H* dx, hipStream_t s) {
  if (n_rows > 0) k_sender_reduce<T, H><<<n_rows, 128, 0, s>>>(n_rows, sptr, sidx, dxe, width, dx);
}
template <typename T>
void launch_ghost_fold(int n_local, const int* gptr, const T* dx_ext, T* dx, int width, hipStream_t s) {
  if (n_local > 0) k_ghost_fold<T><<<n_local, 128, 0, s>>>(n_local, gptr, dx_ext, dx, width);
}
template <typename T>
void launch_dY_reduce(int64_t E, int n_tasks, int NY, const T* part, T* dY, bool accumulate,
                      hipStream_t s) {
  if (E > 0)
    k_dY_reduce<T><<<nblk(E * NY, 256), 256, 0, s>>>(E, n_tasks, NY, part, dY, accumulate ? 1 : 0);
}
void launch_forces(int n_local, const int* row_ptr, const int* sptr, const int* sidx, const int* gptr,
                   const double* g, double* F, hipStream_t s) {
  if (n_local > 0) k_forces<<<nblk(n_local, 4), 256, 0, s>>>(n_local, row_ptr, sptr, sidx, gptr, g, F);
}
void launch_seg_energy(int nchunks, const int* chunks, const double* atom_e, double* partial,
                       hipStream_t s) {
  if (nchunks > 0) k_seg_energy<<<nchunks, kRedThreads, 0, s>>>(chunks, atom_e, partial);
}
void launch_seg_virial(int nchunks, const int* chunks, const int* recv, const int* src,
                       const double* pos_ext, const double* g, double* partial, hipStream_t s) {
  if (nchunks > 0) k_seg_virial<<<nchunks, kRedThreads, 0, s>>>(chunks, recv, src, pos_ext, g, partial);
}
void launch_seg_finalize(int B, const int* first, const double* partial, int width, double* out,
                         const double* gscale, hipStream_t s) {
  if (B > 0)
    k_seg_finalize<<<nblk((int64_t)B * width, 128), 128, 0, s>>>(B, first, partial, width, out, gscale);
}
void launch_unpermute(int n, const int* order, const double* in_rows, int width, double* out_rows,
                      const double* gscale, const int* sid_orig, int regions_per_struct,
                      hipStream_t s) {
  if (n > 0)
    k_unpermute<<<nblk(n, 256), 256, 0, s>>>(n, order, in_rows, width, out_rows, gscale, sid_orig,
                                             regions_per_struct);
}

#define SN_INST(T)                                                                                \
  template void launch_embed<T>(int, const int*, const T*, int, T*, int, hipStream_t);            \
  template void launch_ghost_refresh<T>(int, int, const int*, T*, int, hipStream_t);              \
  template void launch_gate_fwd<T>(int, bool, IrrepLayout, IrrepLayout, const T*, T*, T,          \
                                   hipStream_t);                                                  \
  template void launch_gate_bwd<T, T>(int, bool, IrrepLayout, IrrepLayout, const T*, const T*,    \
                                      T*, T, hipStream_t);                                        \
  template void launch_readout<T>(int, const T*, int, const double*, int, double, const double*,  \
                                  const int*, double*, hipStream_t);                              \
  template void launch_fill_rows<T>(int, const double*, int, double, T*, int, hipStream_t);       \
  template void launch_sender_reduce<T, T>(int, const int*, const int*, const T*, int, T*,        \
                                           hipStream_t);                                          \
  template void launch_ghost_fold<T>(int, const int*, const T*, T*, int, hipStream_t);            \
  template void launch_dY_reduce<T>(int64_t, int, int, const T*, T*, bool, hipStream_t);
SN_INST(float)
SN_INST(double)
#undef SN_INST
// bfloat16 storage of sender features and per-edge sender gradient rows
template void launch_ghost_refresh<bf16_t>(int, int, const int*, bf16_t*, int, hipStream_t);
// float64 forward node state with float32 node gradients (FP32 form)
template void launch_gate_bwd<double, float>(int, bool, IrrepLayout, IrrepLayout, const double*,
                                             const float*, float*, double, hipStream_t);
template void launch_sender_reduce<bf16_t, float>(int, const int*, const int*, const bf16_t*, int,
                                                  float*, hipStream_t);

}  // namespace sn
