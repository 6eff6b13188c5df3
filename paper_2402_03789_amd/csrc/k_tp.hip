// Tensor-product convolution (the message function of the NequIP
// interaction block, paper eq 3 and section 2.2) and its adjoint (eq 7).
//
// For edge e (receiver i, sender s), path p = (l1, l2, l3) and channel u:
//   q[p, u, m3] = w_e[p, u] sum_{m1, m2} C^p[m1, m2, m3] x_s[l1][u, m1] Y_e^{l2}[m2]
//   M_i = (1 / k_avg) sum_{e -> i} q        (section 5.1 normalisation)
// computed as A^p_e[m1][m3] = sum_m2 C^p[m1][m2][m3] Y^{l2}_e[m2] (once per edge,
// in LDS) followed by per-channel contractions.
//
// Work decomposition (MI355X-native): one 64-lane wavefront per (receiver,
// task); a task is one input degree l1 and up to 64 of its channels.  When a
// degree has fewer than 64 channels, the wave processes 64/cpt edges at once
// (lanes = channel x edge slot) and the slots are combined with cross-lane
// shuffles at the end.  Every receiver's edges are contiguous (receiver-sorted
// CSR), so the message sum is a register accumulation with a single write:
// no atomics.  The CG coefficients are compile-time constants (generated), so
// only their nonzeros become instructions.
//
// The adjoint uses dE/dq = G / k_avg with G = dE/dM of the receiver (a
// register-resident row per lane) and produces, per edge:
//   dE/dw[p,u] = sum_m3 G[p,u,m3] t[p,u,m3],  t = x A
//   dE/dx_s[u, m1] (per-edge row, reduced over senders by a separate pass)
//   dE/dY[m2] = sum_{p,u} sum C[m1,m2,m3] x[u,m1] w[p,u] G[p,u,m3]  (cross-lane sum)
#include "kernels.h"
#include "cg_tables.h"

#include <utility>

namespace sn {

template <int L1, int LSH, int L3MAX, bool SO>
struct PathList {
  static constexpr int count() {
    int c = 0;
    for (int l2 = 0; l2 <= LSH; ++l2)
      for (int l3 = (L1 > l2 ? L1 - l2 : l2 - L1); l3 <= (L1 + l2 < L3MAX ? L1 + l2 : L3MAX); ++l3)
        if (!SO || l3 == 0) ++c;
    return c;
  }
  static constexpr int get(int p, int which) {
    int c = 0;
    for (int l2 = 0; l2 <= LSH; ++l2)
      for (int l3 = (L1 > l2 ? L1 - l2 : l2 - L1); l3 <= (L1 + l2 < L3MAX ? L1 + l2 : L3MAX); ++l3)
        if (!SO || l3 == 0) {
          if (c == p) return which == 0 ? l2 : l3;
          ++c;
        }
    return -1;
  }
  static constexpr int l2(int p) { return get(p, 0); }
  static constexpr int l3(int p) { return get(p, 1); }
  static constexpr int aoff(int p) {  // offset of A^p in the per-edge table
    int o = 0;
    for (int q = 0; q < p; ++q) o += (2 * L1 + 1) * (2 * l3(q) + 1);
    return o;
  }
  static constexpr int ooff(int p) {  // offset of path p's outputs in a lane's accumulators
    int o = 0;
    for (int q = 0; q < p; ++q) o += 2 * l3(q) + 1;
    return o;
  }
  static constexpr int NA = aoff(count());
  static constexpr int NOUT = ooff(count());
};

template <class F, int... I>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

struct TPArgs {
  const int* row_ptr;
  const int* src;
  int Dx, xoff, mul, cpt;
  int P, woff;
  int Dm;
  int mo[8];
  int mw[8];
  int task_base, n_tasks_total, NY;
};

// Build A^p for the edge e into a[], from Y_e (compile-time CG terms).
template <typename T, int L1, class PL>
__device__ inline void build_A(const T* __restrict__ Ye, T* a) {
#pragma unroll
  for (int q = 0; q < PL::NA; ++q) a[q] = T(0);
  static_for<PL::count()>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr int l2 = PL::l2(p), l3 = PL::l3(p);
    constexpr int D3 = 2 * l3 + 1;
    constexpr int ao = PL::aoff(p);
    CG<L1, l2, l3>::each([&](int m1, int m2, int m3, double c) {
      a[ao + m1 * D3 + m3] += T(c) * Ye[l2 * l2 + m2];
    });
  });
}

template <typename T, int L1, int LSH, int L3MAX, bool SO, int CH>
__global__ __launch_bounds__(64) void k_tp_fwd(TPArgs g, const T* __restrict__ Y,
                                                const T* __restrict__ x, const T* __restrict__ w,
                                                T* __restrict__ M, T inv_k) {
  using PL = PathList<L1, LSH, L3MAX, SO>;
  constexpr int NP = PL::count();
  constexpr int D1 = 2 * L1 + 1;
  constexpr int NA = PL::NA;
  constexpr int NYc = (LSH + 1) * (LSH + 1);
  __shared__ T sA[CH][NA + 1];
  __shared__ int sSrc[CH];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int cpt = g.cpt;
  const int EI = kWave / cpt;
  const int ei = lane / cpt;
  const int u = blockIdx.y * cpt + (lane % cpt);
  const bool valid = u < g.mul;
  T acc[PL::NOUT];
#pragma unroll
  for (int q = 0; q < PL::NOUT; ++q) acc[q] = T(0);
  const int beg = g.row_ptr[i], end = g.row_ptr[i + 1];
  for (int c0 = beg; c0 < end; c0 += CH) {
    const int n = min(CH, end - c0);
    for (int j = lane; j < n; j += kWave) {
      const int64_t e = c0 + j;
      T Ye[NYc];
#pragma unroll
      for (int q = 0; q < NYc; ++q) Ye[q] = Y[e * g.NY + q];
      T a[NA];
      build_A<T, L1, PL>(Ye, a);
#pragma unroll
      for (int q = 0; q < NA; ++q) sA[j][q] = a[q];
      sSrc[j] = g.src[e];
    }
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += EI) {
      const int j = j0 + ei;
      if (j < n && valid) {
        const int64_t e = c0 + j;
        const int s = sSrc[j];
        T xv[D1];
#pragma unroll
        for (int m1 = 0; m1 < D1; ++m1) xv[m1] = x[(int64_t)s * g.Dx + g.xoff + m1 * g.mul + u];
        static_for<NP>([&](auto P) {
          constexpr int p = decltype(P)::value;
          constexpr int D3 = 2 * PL::l3(p) + 1;
          constexpr int ao = PL::aoff(p), oo = PL::ooff(p);
          const T wv = w[e * g.P + g.woff + p * g.mul + u];
#pragma unroll
          for (int m3 = 0; m3 < D3; ++m3) {
            T t = T(0);
#pragma unroll
            for (int m1 = 0; m1 < D1; ++m1) t += xv[m1] * sA[j][ao + m1 * D3 + m3];
            acc[oo + m3] += wv * t;
          }
        });
      }
    }
    __syncthreads();
  }
  for (int off = cpt; off < kWave; off <<= 1) {
#pragma unroll
    for (int q = 0; q < PL::NOUT; ++q) acc[q] += __shfl_xor(acc[q], off);
  }
  if (ei == 0 && valid) {
    static_for<NP>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr int D3 = 2 * PL::l3(p) + 1;
      constexpr int oo = PL::ooff(p);
#pragma unroll
      for (int m3 = 0; m3 < D3; ++m3)
        M[(int64_t)i * g.Dm + g.mo[p] + m3 * g.mw[p] + u] = acc[oo + m3] * inv_k;
    });
  }
}

template <typename T, int L1, int LSH, int L3MAX, bool SO, int CH, bool WRITE_DX>
__global__ __launch_bounds__(64) void k_tp_bwd(TPArgs g, const T* __restrict__ Y,
                                                const T* __restrict__ x, const T* __restrict__ w,
                                                const T* __restrict__ G, T* __restrict__ dw,
                                                T* __restrict__ dxe, T* __restrict__ dYpart) {
  using PL = PathList<L1, LSH, L3MAX, SO>;
  constexpr int NP = PL::count();
  constexpr int D1 = 2 * L1 + 1;
  constexpr int NA = PL::NA;
  constexpr int NYc = (LSH + 1) * (LSH + 1);
  __shared__ T sA[CH][NA + 1];
  __shared__ int sSrc[CH];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int cpt = g.cpt;
  const int EI = kWave / cpt;
  const int ei = lane / cpt;
  const int uu = lane % cpt;
  const int u = blockIdx.y * cpt + uu;
  const bool valid = u < g.mul;
  const int task = g.task_base + blockIdx.y;
  T gin[PL::NOUT];
  static_for<NP>([&](auto P) {
    constexpr int p = decltype(P)::value;
    constexpr int D3 = 2 * PL::l3(p) + 1;
    constexpr int oo = PL::ooff(p);
#pragma unroll
    for (int m3 = 0; m3 < D3; ++m3)
      gin[oo + m3] = valid ? G[(int64_t)i * g.Dm + g.mo[p] + m3 * g.mw[p] + u] : T(0);
  });
  const int beg = g.row_ptr[i], end = g.row_ptr[i + 1];
  for (int c0 = beg; c0 < end; c0 += CH) {
    const int n = min(CH, end - c0);
    for (int j = lane; j < n; j += kWave) {
      const int64_t e = c0 + j;
      T Ye[NYc];
#pragma unroll
      for (int q = 0; q < NYc; ++q) Ye[q] = Y[e * g.NY + q];
      T a[NA];
      build_A<T, L1, PL>(Ye, a);
#pragma unroll
      for (int q = 0; q < NA; ++q) sA[j][q] = a[q];
      sSrc[j] = g.src[e];
    }
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += EI) {
      const int j = j0 + ei;
      const bool active = j < n;
      T dYl[NYc];
#pragma unroll
      for (int q = 0; q < NYc; ++q) dYl[q] = T(0);
      if (active && valid) {
        const int64_t e = c0 + j;
        const int s = sSrc[j];
        T xv[D1], dxv[D1];
#pragma unroll
        for (int m1 = 0; m1 < D1; ++m1) {
          xv[m1] = x[(int64_t)s * g.Dx + g.xoff + m1 * g.mul + u];
          dxv[m1] = T(0);
        }
        static_for<NP>([&](auto P) {
          constexpr int p = decltype(P)::value;
          constexpr int l2 = PL::l2(p), l3 = PL::l3(p);
          constexpr int D3 = 2 * l3 + 1;
          constexpr int ao = PL::aoff(p), oo = PL::ooff(p);
          const int64_t widx = e * g.P + g.woff + p * g.mul + u;
          const T wv = w[widx];
          T dwv = T(0);
          T gg[D3];
#pragma unroll
          for (int m3 = 0; m3 < D3; ++m3) {
            T t = T(0);
#pragma unroll
            for (int m1 = 0; m1 < D1; ++m1) t += xv[m1] * sA[j][ao + m1 * D3 + m3];
            dwv += gin[oo + m3] * t;
            gg[m3] = wv * gin[oo + m3];
          }
          dw[widx] = dwv;
          if (WRITE_DX) {
#pragma unroll
            for (int m1 = 0; m1 < D1; ++m1) {
              T v = T(0);
#pragma unroll
              for (int m3 = 0; m3 < D3; ++m3) v += sA[j][ao + m1 * D3 + m3] * gg[m3];
              dxv[m1] += v;
            }
          }
          CG<L1, l2, l3>::each([&](int m1, int m2, int m3, double c) {
            dYl[l2 * l2 + m2] += T(c) * xv[m1] * gg[m3];
          });
        });
        if (WRITE_DX) {
#pragma unroll
          for (int m1 = 0; m1 < D1; ++m1) dxe[e * g.Dx + g.xoff + m1 * g.mul + u] = dxv[m1];
        }
      }
      for (int off = 1; off < cpt; off <<= 1) {
#pragma unroll
        for (int q = 0; q < NYc; ++q) dYl[q] += __shfl_xor(dYl[q], off);
      }
      if (uu == 0 && active) {
        const int64_t e = c0 + j;
        T* dst = dYpart + (e * g.n_tasks_total + task) * g.NY;
#pragma unroll
        for (int q = 0; q < NYc; ++q) dst[q] = dYl[q];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ dispatch
template <typename T>
struct TPChunk { static constexpr int value = 64; };
template <>
struct TPChunk<double> { static constexpr int value = 32; };

template <typename T, int L1, int LSH, int L3MAX, bool SO>
static void fwd_one(const TPArgs& a, int n_recv, int n_tasks, const T* Y, const T* x, const T* w,
                    T* M, T inv_k, hipStream_t s) {
  dim3 grid(n_recv, n_tasks);
  k_tp_fwd<T, L1, LSH, L3MAX, SO, TPChunk<T>::value><<<grid, kWave, 0, s>>>(a, Y, x, w, M, inv_k);
}
template <typename T, int L1, int LSH, int L3MAX, bool SO>
static void bwd_one(const TPArgs& a, int n_recv, int n_tasks, const T* Y, const T* x, const T* w,
                    const T* G, T* dw, T* dxe, T* dYp, hipStream_t s) {
  dim3 grid(n_recv, n_tasks);
  if (dxe)
    k_tp_bwd<T, L1, LSH, L3MAX, SO, TPChunk<T>::value, true>
        <<<grid, kWave, 0, s>>>(a, Y, x, w, G, dw, dxe, dYp);
  else
    k_tp_bwd<T, L1, LSH, L3MAX, SO, TPChunk<T>::value, false>
        <<<grid, kWave, 0, s>>>(a, Y, x, w, G, dw, dxe, dYp);
}

// (lsh, lmax) in {(1,1), (2,2)}; l1 <= lmax; scalar-only flag
template <typename T, bool FWD>
static void dispatch(const TPLayer& L, int l1, const TPArgs& a, int n_recv, int n_tasks,
                     const T* Y, const T* x, const T* w, T* M, T inv_k, const T* G, T* dw, T* dxe,
                     T* dYp, hipStream_t s) {
#define SN_TP_CASE(LL1, LSH, LMX, SO)                                                    \
  if (l1 == LL1 && L.lsh == LSH && L.lmax == LMX && L.scalar_only == SO) {               \
    if (FWD)                                                                             \
      fwd_one<T, LL1, LSH, LMX, SO>(a, n_recv, n_tasks, Y, x, w, M, inv_k, s);           \
    else                                                                                 \
      bwd_one<T, LL1, LSH, LMX, SO>(a, n_recv, n_tasks, Y, x, w, G, dw, dxe, dYp, s);    \
    return;                                                                              \
  }
  SN_TP_CASE(0, 1, 1, false) SN_TP_CASE(1, 1, 1, false)
  SN_TP_CASE(0, 1, 1, true) SN_TP_CASE(1, 1, 1, true)
  SN_TP_CASE(0, 2, 2, false) SN_TP_CASE(1, 2, 2, false) SN_TP_CASE(2, 2, 2, false)
  SN_TP_CASE(0, 2, 2, true) SN_TP_CASE(1, 2, 2, true) SN_TP_CASE(2, 2, 2, true)
#undef SN_TP_CASE
}

template <typename T>
static void run(const TPLayer& L, bool fwd, int n_recv, const int* row_ptr, const int* src,
                const T* Y, const T* x, const T* w, T* M, T inv_k, const T* G, T* dw, T* dxe,
                T* dYp, hipStream_t s) {
  if (n_recv <= 0) return;
  int t = 0;
  for (int l1 = 0; l1 <= L.lmax; ++l1) {
    int nt = 0, cpt = 0;
    for (int k = 0; k < L.n_tasks; ++k)
      if (L.tasks[k].l1 == l1) { ++nt; cpt = L.tasks[k].cpt; }
    if (nt == 0) continue;
    TPArgs a{};
    a.row_ptr = row_ptr;
    a.src = src;
    a.Dx = L.xin.width;
    a.xoff = L.xin.off[l1];
    a.mul = L.xin.mul[l1];
    a.cpt = cpt;
    a.P = L.P;
    a.woff = L.woff[l1];
    a.Dm = L.Dm;
    for (int p = 0; p < 8; ++p) { a.mo[p] = L.mo[l1][p]; a.mw[p] = L.mw[l1][p]; }
    a.task_base = t;
    a.n_tasks_total = L.n_tasks;
    a.NY = L.NY;
    if (fwd)
      dispatch<T, true>(L, l1, a, n_recv, nt, Y, x, w, M, inv_k, nullptr, nullptr, nullptr, nullptr, s);
    else
      dispatch<T, false>(L, l1, a, n_recv, nt, Y, x, w, nullptr, inv_k, G, dw, dxe, dYp, s);
    t += nt;
  }
}

template <typename T>
void launch_tp_fwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src, const T* Y,
                   const T* x, const T* w, T* M, T inv_k, hipStream_t s) {
  run<T>(L, true, n_recv, row_ptr, src, Y, x, w, M, inv_k, nullptr, nullptr, nullptr, nullptr, s);
}
template <typename T>
void launch_tp_bwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src, const T* Y,
                   const T* x, const T* w, const T* G, T* dw, T* dxe, T* dYpart, hipStream_t s) {
  run<T>(L, false, n_recv, row_ptr, src, Y, x, w, nullptr, T(0), G, dw, dxe, dYpart, s);
}

template void launch_tp_fwd<float>(const TPLayer&, int, const int*, const int*, const float*,
                                   const float*, const float*, float*, float, hipStream_t);
template void launch_tp_fwd<double>(const TPLayer&, int, const int*, const int*, const double*,
                                    const double*, const double*, double*, double, hipStream_t);
template void launch_tp_bwd<float>(const TPLayer&, int, const int*, const int*, const float*,
                                   const float*, const float*, const float*, float*, float*, float*,
                                   hipStream_t);
template void launch_tp_bwd<double>(const TPLayer&, int, const int*, const int*, const double*,
                                    const double*, const double*, const double*, double*, double*,
                                    double*, hipStream_t);

}  // namespace sn
