// Tensor-product convolution (the message function of the NequIP
// interaction block, paper eq 3 and section 2.2) and its adjoint (eq 7).
//
// For edge e (receiver i, sender s), path p = (l1, l2, l3) and channel u:
//   q[p, u, m3] = w_e[p, u] sum_{m1, m2} C^p[m1, m2, m3] x_s[l1][u, m1] Y_e^{l2}[m2]
//   M_i = (1 / k_avg) sum_{e -> i} q        (section 5.1 normalisation)
// The CG coefficients are compile-time constants produced by the generator, so
// only their nonzeros become instructions and no coupling table occupies LDS.
//
// Work decomposition (MI355X-native): one kernel per input degree l1 (so each
// gets its own register budget), one 64-lane wavefront per receiver and one
// wave per block (measured faster than two or four per block: the waves of a
// launch are placed one by one).  A wave covers the degree's channels with lanes (two
// channels per lane for a 128-channel scalar block: the adjacent pair 2u, 2u + 1, so every
// value moves as one 2-wide access, where the row offsets allow); a degree with fewer than
// 64 channels processes 64/cpt edges at once (lanes = channel x edge slot) and
// combines the slots with cross-lane shuffles at the end.  The radial weights
// are read through the edge's pair index (an edge and its reverse share them).  Every receiver's
// edges are contiguous (receiver-sorted CSR), so the message sum is a register
// accumulation followed by a single write: no atomics.
//
// The adjoint uses dE/dq = G / k_avg with G = dE/dM of the receiver (register
// resident per lane) and produces, per edge:
//   dE/dw[p,u] = sum_m3 G[p,u,m3] t[p,u,m3],  t[m3] = sum C x[m1] Y[m2]
//     (stored pair-major: the two edges of a pair write adjacent rows, so the MLP
//     adjoint streams them in pair order)
//   dE/dx_s[u, m1] (a per-edge row, reduced over senders by a separate pass)
//   dE/dY[m2] = sum_{p,u} sum C[m1,m2,m3] x[u,m1] w[p,u] G[p,u,m3]
// The channel sum of dE/dY runs inside each wave (DPP exchanges within 16-lane rows,
// shuffles across rows); the per-degree kernels add their shares to dE/dY one after
// another (fixed order).  Both directions are compiled for slot widths of 64 and 32
// lanes (fewer registers, so more waves per SIMD) besides the general runtime width.
#pragma once

#include "kernels.h"
#include "cg_tables.h"

#include <stdexcept>
#include <type_traits>
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
  static constexpr int ooff(int p) {  // offset of path p's outputs in a lane's accumulators
    int o = 0;
    for (int q = 0; q < p; ++q) o += 2 * l3(q) + 1;
    return o;
  }
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

// Two consecutive channels of one row as one access, for lanes that own a channel pair
// (PAIR kernels: 2 u, 2 u + 1 on lane slot u).  The row offsets are even, so the access is
// aligned to its size.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ inline void ld2(const float* p, T& a, T& b) {
  const f32x2 v = *reinterpret_cast<const f32x2*>(p);
  a = (T)v[0];
  b = (T)v[1];
}
template <typename T>
__device__ inline void ld2(const double* p, T& a, T& b) {
  const f64x2 v = *reinterpret_cast<const f64x2*>(p);
  a = (T)v[0];
  b = (T)v[1];
}
template <typename T>
__device__ inline void ld2(const bf16_t* p, T& a, T& b) {
  const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
  a = (T)__uint_as_float(v << 16);
  b = (T)__uint_as_float(v & 0xffff0000u);
}
template <typename T>
__device__ inline void st2(float* p, T a, T b) {
  *reinterpret_cast<f32x2*>(p) = f32x2{sstore<float>(a), sstore<float>(b)};
}
template <typename T>
__device__ inline void st2(double* p, T a, T b) {
  *reinterpret_cast<f64x2*>(p) = f64x2{sstore<double>(a), sstore<double>(b)};
}
template <typename T>
__device__ inline void st2(bf16_t* p, T a, T b) {
  *reinterpret_cast<uint32_t*>(p) =
      (uint32_t)sstore<bf16_t>(a).u | ((uint32_t)sstore<bf16_t>(b).u << 16);
}

// Per-degree arguments of one interaction block.
struct TPDeg {
  int xoff, mul, cpt, cpl;  // feature block offset, channels, lanes per edge slot, channels per lane
  int woff;                 // first radial weight of the paths with this l1
  int mo[kMaxPathsL1], mw[kMaxPathsL1];  // per path: offset in the message row, width of its l3 block
};

struct TPArgs {
  const int* row_ptr;
  const int* src;
  const int* pidx;  // 2 p + side: pair p holds the shared radial weights, 2 p + side the dE/dw row
  int n_recv;
  int split_log;    // adjoint: 2^split_log waves share a receiver's edges (contiguous slices)
  int Dx, P, Dm, NY;
  TPDeg d;
};

// channels per lane: two for a 128-channel scalar block, one otherwise
template <int L1>
struct CPL { static constexpr int value = L1 == 0 ? 2 : 1; };

constexpr int kRecvPerBlock = 1;  // receivers (waves) per block

// t[m3] = sum_{m1,m2} C[m1,m2,m3] x[m1] Y[m2] of one path (l1, l2, l3) for one edge and one
// channel; each path's t is formed where it is used, so at most 2 l3 + 1 of them are live
template <typename T, int L1, int L2, int L3>
__device__ inline void tp_path(const T* xv, const T* Ye, T (&t)[2 * L3 + 1]) {
#pragma unroll
  for (int q = 0; q < 2 * L3 + 1; ++q) t[q] = T(0);
  CG<L1, L2, L3>::each([&](int m1, int m2, int m3, double c) {
    t[m3] += T(c) * (xv[m1] * Ye[L2 * L2 + m2]);
  });
}

// Operands of one edge for one lane.  The edge loop is software-pipelined through a
// ring of R operand sets (static slots, the loop unrolled by R): indices are loaded 2R-1
// iterations ahead of their edge's compute and operands R-1 ahead.  Every load is
// unconditional from a valid address (edge index clamped to the receiver's last edge,
// channel clamped to 0 on idle lanes) and the values are masked where they are used: a
// load under a branch makes the compiler wait for it, and for every other load in
// flight, inside that branch, which would undo the prefetch.
template <typename T, int D1, int NP, int NYc, int KC>
struct EdgeOps {
  T Y[NYc];
  T x[KC][D1];
  T w[KC][NP];
  T dyo;  // adjoint: this edge's earlier share of dE/dY (the lane's value)
  int p;  // pair slot 2 p + side
};
struct EdgeIdx {
  int s, p;
};

template <typename T, typename S, int D1, int NP, int NYc, int KC, bool PAIR = false>
__device__ inline void load_edge(const TPArgs& g, const TPDeg& a, const int (&uc)[KC], int64_t e,
                                 const EdgeIdx& ix, const T* __restrict__ Y, const S* __restrict__ x,
                                 const S* __restrict__ w, EdgeOps<T, D1, NP, NYc, KC>& o) {
#pragma unroll
  for (int q = 0; q < NYc; ++q) o.Y[q] = Y[e * g.NY + q];
  const int64_t wrow = (int64_t)(ix.p >> 1) * g.P + a.woff;
  const int64_t xrow = (int64_t)ix.s * g.Dx + a.xoff;
  if constexpr (PAIR) {  // uc[1] = uc[0] + 1
#pragma unroll
    for (int m1 = 0; m1 < D1; ++m1) ld2(&x[xrow + m1 * a.mul + uc[0]], o.x[0][m1], o.x[1][m1]);
#pragma unroll
    for (int p = 0; p < NP; ++p) ld2(&w[wrow + p * a.mul + uc[0]], o.w[0][p], o.w[1][p]);
    o.p = ix.p;
    return;
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
#pragma unroll
    for (int m1 = 0; m1 < D1; ++m1) o.x[c][m1] = (T)sload(x[xrow + m1 * a.mul + uc[c]]);
#pragma unroll
    for (int p = 0; p < NP; ++p) o.w[c][p] = (T)sload(w[wrow + p * a.mul + uc[c]]);
  }
  o.p = ix.p;
}

// Runs compute(k, ops) for every edge iteration k < n_it of a receiver through the ring
// pipeline; extra(k, ops) adds per-edge loads of the caller (issued with the operands).
template <int R, typename OPS, class Load, class Compute>
__device__ inline void edge_pipeline(const TPArgs& g, int beg, int end, int EI, int ei, int n_it,
                                     Load&& load, Compute&& compute) {
  const int deg = end - beg;
  auto edge_of = [&](int kl) { return beg + min(kl * EI + ei, deg - 1); };
  auto load_idx = [&](int kl, EdgeIdx& d) {
    const int e = edge_of(kl);
    d.s = g.src[e];
    d.p = g.pidx[e];
  };
  EdgeIdx ix[R];
  OPS ops[R];
  static_for<R>([&](auto J) { load_idx(decltype(J)::value, ix[decltype(J)::value]); });
  static_for<R - 1>([&](auto J) {
    constexpr int j = decltype(J)::value;
    load(edge_of(j), ix[j], ops[j]);
    load_idx(j + R, ix[j]);
  });
  for (int k = 0; k < n_it; k += R) {
    static_for<R>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr int jf = (j + R - 1) % R;
      const int kk = k + j;
      load(edge_of(kk + R - 1), ix[jf], ops[jf]);
      load_idx(kk + 2 * R - 1, ix[jf]);
      if (kk < n_it) compute(kk, ops[j]);
    });
  }
}

template <typename T, typename S, int L1, int LSH, int L3MAX, bool SO, int CPT, bool PAIR = false>
__global__ __launch_bounds__(256) void k_tp_fwd(TPArgs g, const T* __restrict__ Y,
                                                 const S* __restrict__ x, const S* __restrict__ w,
                                                 S* __restrict__ M, T inv_k) {
  using PL = PathList<L1, LSH, L3MAX, SO>;
  constexpr int NP = PL::count();
  constexpr int D1 = 2 * L1 + 1;
  constexpr int NYc = (LSH + 1) * (LSH + 1);
  constexpr int NO = PL::NOUT;
  constexpr int KC = CPL<L1>::value;
  // receiver of this wave (wave-uniform; kept in a scalar register)
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kRecvPerBlock + (threadIdx.x >> 6));
  if (i >= g.n_recv) return;
  const TPDeg& a = g.d;
  const int lane = threadIdx.x & 63;
  // lanes per edge slot: a compile-time 64 or 32 for the common widths (a 64-lane slot makes
  // every edge index wave-uniform), else the runtime value
  const int cpt = CPT ? CPT : a.cpt, EI = kWave / cpt, ei = lane / cpt, uu = lane % cpt;
  T acc[KC][NO];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int q = 0; q < NO; ++q) acc[c][q] = T(0);
  const int beg = g.row_ptr[i], end = g.row_ptr[i + 1];
  const int n_it = (end - beg + EI - 1) / EI;
  static_assert(!PAIR || KC == 2, "channel pairs need two channels per lane");
  int uc[KC];
  bool ok[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int u = PAIR ? 2 * uu + c : uu + c * cpt;
    ok[c] = c < a.cpl && u < a.mul;
    uc[c] = ok[c] ? u : (PAIR ? c : 0);
  }
  using Ops = EdgeOps<T, D1, NP, NYc, KC>;
  if (n_it > 0)
    edge_pipeline<(CPT == 32 ? 3 : 4), Ops>(
        g, beg, end, EI, ei, n_it,
        [&](int e, const EdgeIdx& ix, Ops& o) {
          load_edge<T, S, D1, NP, NYc, KC, PAIR>(g, a, uc, e, ix, Y, x, w, o);
        },
        [&](int k, const Ops& cur) {
          const bool active = beg + k * EI + ei < end;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            static_for<NP>([&](auto P) {
              constexpr int p = decltype(P)::value;
              constexpr int l3 = PL::l3(p);
              constexpr int oo = PL::ooff(p);
              T t[2 * l3 + 1];
              tp_path<T, L1, PL::l2(p), l3>(cur.x[c], cur.Y, t);
              const T wv = (active && ok[c]) ? cur.w[c][p] : T(0);
#pragma unroll
              for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) acc[c][oo + m3] += wv * t[m3];
            });
          }
        });
  for (int off = cpt; off < kWave; off <<= 1) {
#pragma unroll
    for (int c = 0; c < KC; ++c)
#pragma unroll
      for (int q = 0; q < NO; ++q) acc[c][q] += __shfl_xor(acc[c][q], off);
  }
  if (ei != 0) return;
  if constexpr (PAIR) {
    if (2 * uu >= a.mul) return;  // both channels of the pair or neither (mul is even)
    const int u = 2 * uu;
    static_for<NP>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr int D3 = 2 * PL::l3(p) + 1;
      constexpr int oo = PL::ooff(p);
#pragma unroll
      for (int m3 = 0; m3 < D3; ++m3)
        st2(&M[(int64_t)i * g.Dm + a.mo[p] + m3 * a.mw[p] + u], acc[0][oo + m3] * inv_k,
            acc[1][oo + m3] * inv_k);
    });
    return;
  }
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int u = uu + c * cpt;
    if (c >= a.cpl || u >= a.mul) break;
    static_for<NP>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr int D3 = 2 * PL::l3(p) + 1;
      constexpr int oo = PL::ooff(p);
#pragma unroll
      for (int m3 = 0; m3 < D3; ++m3)
        M[(int64_t)i * g.Dm + a.mo[p] + m3 * a.mw[p] + u] = sstore<S>(acc[c][oo + m3] * inv_k);
    });
  }
}

// Sum over the cpt lanes of an edge slot of NV values per lane (NV a power of two, the
// first NYc of them meaningful), as a transposed butterfly: at each of the first
// S = min(log2 NV, log2 cpt) stages a lane keeps one half of its values, receives its
// partner's partial sums of that half and sends the other half, so the value count
// halves per stage (NV/2 shuffles instead of NV); the remaining stages are plain.
// Afterwards the lane holds the complete sums of values j0 .. j0 + (NV >> S) - 1, where
// j0 = slot_first_value(lane, cpt), and lanes whose low bits (cpt >> S) - 1 are zero
// hold distinct value groups.
template <int NV>
__device__ inline int slot_first_value(int lane, int cpt) {
  int j0 = 0, o = cpt >> 1, h = NV >> 1;
  while (o > 0 && h > 0) {
    if (lane & o) j0 += h;
    o >>= 1;
    h >>= 1;
  }
  return j0;
}
template <int NV>
__device__ inline int slot_store_mask(int cpt) {
  int o = cpt, v = NV;
  while (o > 1 && v > 1) {
    o >>= 1;
    v >>= 1;
  }
  return o - 1;  // lanes with (lane & mask) == 0 store
}
template <typename T, int NV>
__device__ inline void slot_reduce(T (&v)[NV], int cpt, int lane) {
  int o = cpt >> 1;
  static_for<NV == 1 ? 0 : (NV == 2 ? 1 : (NV == 4 ? 2 : (NV == 8 ? 3 : 4)))>([&](auto K) {
    constexpr int H = NV >> (decltype(K)::value + 1);
    if (o > 0) {
      const bool hi = (lane & o) != 0;
#pragma unroll
      for (int r = 0; r < H; ++r) {
        const T send = hi ? v[r] : v[r + H];
        const T keep = hi ? v[r + H] : v[r];
        v[r] = keep + __shfl_xor(send, o);
      }
      o >>= 1;
    }
  });
  for (; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
}

// The same transposed reduction for slots of at least 16 lanes, with its exchanges inside
// 16-lane rows done by DPP lane permutations on the adding instruction (no LDS round
// trip): the transposed stages pair lanes i and i ^ 15 (row mirror), i ^ 7 (half-row
// mirror), i ^ 2 and i ^ 1 (quad permutations), in that order, each on the lane-id bit it
// flips highest (3, 2, 1, 0), so that both lanes of a pair hold the same value group; the
// four masks span every lane of a row.  Remaining row bits and the cross-row bits of the
// slot (16, 32) are plain stages on one value.  Afterwards lane l holds the complete sum
// of value slot_first_value_rows<NV>(l), identical in every row of the slot.
constexpr int kDppRowMirror = 0x140, kDppHalfMirror = 0x141;
constexpr int kDppXor2 = 0x4E, kDppXor1 = 0xB1;  // quad_perm [2,3,0,1] and [1,0,3,2]
template <int CTRL>
__device__ inline float dpp_get(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_get(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int K>
struct RowStage;  // stage K: DPP control and the lane-id bit it flips highest
template <> struct RowStage<0> { static constexpr int ctrl = kDppRowMirror, bit = 8; };
template <> struct RowStage<1> { static constexpr int ctrl = kDppHalfMirror, bit = 4; };
template <> struct RowStage<2> { static constexpr int ctrl = kDppXor2, bit = 2; };
template <> struct RowStage<3> { static constexpr int ctrl = kDppXor1, bit = 1; };
template <int NV>
constexpr int log2_nv() { return NV == 1 ? 0 : (NV == 2 ? 1 : (NV == 4 ? 2 : (NV == 8 ? 3 : 4))); }
template <int NV>
__device__ inline int slot_first_value_rows(int lane) {
  int j0 = 0;
  static_for<log2_nv<NV>()>([&](auto K) {
    constexpr int k = decltype(K)::value;
    if (lane & RowStage<k>::bit) j0 += NV >> (k + 1);
  });
  return j0;
}
template <typename T, int NV>
__device__ inline void slot_reduce_rows(T (&v)[NV], int cpt, int lane) {
  constexpr int S = log2_nv<NV>();
  static_for<S>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int H = NV >> (k + 1);
    const bool hi = (lane & RowStage<k>::bit) != 0;
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const T send = hi ? v[r] : v[r + H];
      const T keep = hi ? v[r + H] : v[r];
      v[r] = keep + dpp_get<RowStage<k>::ctrl>(send);
    }
  });
  static_for<4 - S>([&](auto K) {  // the row bits left: plain stages on the one value
    constexpr int k = S + decltype(K)::value;
    v[0] += dpp_get<RowStage<k>::ctrl>(v[0]);
  });
  for (int o = 16; o < cpt; o <<= 1) v[0] += __shfl_xor(v[0], o);
}

// Adjoint of one degree's paths: writes dE/dw (per edge), the per-edge dE/dx rows, and
// adds this degree's share of dE/dY (set instead when accumulate is 0).
template <typename T, typename S, int L1, int LSH, int L3MAX, bool SO, bool WRITE_DX, int CPT,
          bool PAIR = false>
__global__ __launch_bounds__(256) void k_tp_bwd(TPArgs g, const T* __restrict__ Y,
                                                 const S* __restrict__ x, const S* __restrict__ w,
                                                 const S* __restrict__ G, S* __restrict__ dw,
                                                 S* __restrict__ dxe, T* __restrict__ dY,
                                                 int accumulate) {
  using PL = PathList<L1, LSH, L3MAX, SO>;
  constexpr int NP = PL::count();
  constexpr int D1 = 2 * L1 + 1;
  constexpr int NYc = (LSH + 1) * (LSH + 1);
  constexpr int NO = PL::NOUT;
  constexpr int KC = CPL<L1>::value;
  // receiver of this wave (wave-uniform; kept in a scalar register)
  // receiver of this wave and its slice of the receiver's edges (wave-uniform; scalar
  // registers).  Every edge's outputs depend on that edge and G alone, so slices need no
  // combining; small graphs use several waves per receiver to fill the chip.
  const int task = __builtin_amdgcn_readfirstlane(blockIdx.x * kRecvPerBlock + (threadIdx.x >> 6));
  const int i = task >> g.split_log;
  if (i >= g.n_recv) return;
  const TPDeg& a = g.d;
  const int lane = threadIdx.x & 63;
  // lanes per edge slot: a compile-time 64 or 32 for the common widths (a 64-lane slot makes
  // every edge index wave-uniform), else the runtime value
  const int cpt = CPT ? CPT : a.cpt, EI = kWave / cpt, ei = lane / cpt, uu = lane % cpt;
  static_assert(!PAIR || KC == 2, "channel pairs need two channels per lane");
  T gin[KC][NO];
  if constexpr (PAIR) {
    const bool ok = 2 * uu < a.mul;  // both channels of the pair or neither (mul is even)
    const int u = ok ? 2 * uu : 0;
    static_for<NP>([&](auto P) {
      constexpr int p = decltype(P)::value;
      constexpr int D3 = 2 * PL::l3(p) + 1;
      constexpr int oo = PL::ooff(p);
#pragma unroll
      for (int m3 = 0; m3 < D3; ++m3) {
        T g0, g1;
        ld2(&G[(int64_t)i * g.Dm + a.mo[p] + m3 * a.mw[p] + u], g0, g1);
        gin[0][oo + m3] = ok ? g0 : T(0);
        gin[1][oo + m3] = ok ? g1 : T(0);
      }
    });
  } else {
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int u = uu + c * cpt;
      const bool ok = c < a.cpl && u < a.mul;
      static_for<NP>([&](auto P) {
        constexpr int p = decltype(P)::value;
        constexpr int D3 = 2 * PL::l3(p) + 1;
        constexpr int oo = PL::ooff(p);
#pragma unroll
        for (int m3 = 0; m3 < D3; ++m3)
          gin[c][oo + m3] = ok ? (T)sload(G[(int64_t)i * g.Dm + a.mo[p] + m3 * a.mw[p] + u]) : T(0);
      });
    }
  }
  int beg = g.row_ptr[i], end = g.row_ptr[i + 1];
  if (g.split_log) {
    const int len = (end - beg + (1 << g.split_log) - 1) >> g.split_log;
    const int b0 = min(end, beg + (task & ((1 << g.split_log) - 1)) * len);
    end = min(end, b0 + len);
    beg = b0;
  }
  const int n_it = (end - beg + EI - 1) / EI;
  if (n_it == 0) return;
  int uc[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    const int u = PAIR ? 2 * uu + c : uu + c * cpt;
    uc[c] = (c < a.cpl && u < a.mul) ? u : (PAIR ? c : 0);
  }
  // dE/dY: NV = NYc rounded up to a power of two values per lane, reduced per edge slot.
  // With at least NV lanes per slot (every degree of at least NV channels) the transposed
  // butterfly leaves one complete value per storing lane; narrower slots take a plain
  // butterfly and one storing lane.
  constexpr int NV = NYc <= 1 ? 1 : (NYc <= 2 ? 2 : (NYc <= 4 ? 4 : (NYc <= 8 ? 8 : 16)));
  // slots of whole 16-lane rows reduce with DPP row exchanges; narrower ones with shuffles
  const bool rows = cpt >= 16;
  const bool wide = cpt >= NV;
  const int j0 = rows ? slot_first_value_rows<NV>(uu) : (wide ? slot_first_value<NV>(uu, cpt) : 0);
  const bool storer = rows ? uu < 16 && (uu & (16 / NV - 1)) == 0 && j0 < NYc
                           : (wide ? (uu & slot_store_mask<NV>(cpt)) == 0 && j0 < NYc : uu == 0);
  const int jl = min(j0, NYc - 1);
  using Ops = EdgeOps<T, D1, NP, NYc, KC>;
  edge_pipeline<(CPT == 32 ? 2 : 3), Ops>(
      g, beg, end, EI, ei, n_it,
      [&](int e, const EdgeIdx& ix, Ops& o) {
        load_edge<T, S, D1, NP, NYc, KC, PAIR>(g, a, uc, e, ix, Y, x, w, o);
        o.dyo = dY[(int64_t)e * g.NY + jl];  // earlier share of this edge's dE/dY
      },
      [&](int k, const Ops& cur) {
        const int ec = beg + k * EI + ei;
        const bool active = ec < end;
        T dYl[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) dYl[q] = T(0);
        if (active) {
          const int64_t e = ec;
          const int64_t drow = (int64_t)cur.p * g.P + a.woff;  // pair-major dE/dw row
          // PAIR: the pair's dE/dw and dxe values are kept and stored together below
          T dwp[PAIR ? 2 : 1][PAIR ? NP : 1];
          T dxp[PAIR ? 2 : 1][PAIR ? D1 : 1];
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            const int u = PAIR ? 2 * uu + c : uu + c * cpt;
            if (c >= a.cpl || u >= a.mul) break;
            const T* xv = cur.x[c];
            T dxv[D1];
#pragma unroll
            for (int m1 = 0; m1 < D1; ++m1) dxv[m1] = T(0);
            static_for<NP>([&](auto P) {
              constexpr int p = decltype(P)::value;
              constexpr int l2 = PL::l2(p), l3 = PL::l3(p);
              constexpr int D3 = 2 * l3 + 1;
              constexpr int oo = PL::ooff(p);
              T t[D3];
              tp_path<T, L1, l2, l3>(xv, cur.Y, t);
              const T wv = cur.w[c][p];
              T dwv = T(0);
              T gg[D3];
#pragma unroll
              for (int m3 = 0; m3 < D3; ++m3) {
                const T gi = gin[c][oo + m3];
                dwv += gi * t[m3];
                gg[m3] = wv * gi;
              }
              if constexpr (PAIR) dwp[c][p] = dwv;
              else dw[drow + p * a.mul + u] = sstore<S>(dwv);
              CG<L1, l2, l3>::each([&](int m1, int m2, int m3, double cc) {
                if (WRITE_DX) dxv[m1] += T(cc) * (cur.Y[l2 * l2 + m2] * gg[m3]);
                dYl[l2 * l2 + m2] += T(cc) * (xv[m1] * gg[m3]);
              });
            });
            if constexpr (PAIR) {
#pragma unroll
              for (int m1 = 0; m1 < D1; ++m1) dxp[c][m1] = dxv[m1];
            } else if (WRITE_DX) {
#pragma unroll
              for (int m1 = 0; m1 < D1; ++m1)
                dxe[e * g.Dx + a.xoff + m1 * a.mul + u] = sstore<S>(dxv[m1]);
            }
          }
          if constexpr (PAIR) {
            if (2 * uu < a.mul) {  // both channels of the pair (mul is even)
              const int u = 2 * uu;
#pragma unroll
              for (int p = 0; p < NP; ++p) st2(&dw[drow + p * a.mul + u], dwp[0][p], dwp[1][p]);
              if (WRITE_DX) {
#pragma unroll
                for (int m1 = 0; m1 < D1; ++m1)
                  st2(&dxe[e * g.Dx + a.xoff + m1 * a.mul + u], dxp[0][m1], dxp[1][m1]);
              }
            }
          }
        }
        if (rows) {
          slot_reduce_rows<T, NV>(dYl, cpt, lane);
          if (active && storer) dY[(int64_t)ec * g.NY + j0] = (accumulate ? cur.dyo : T(0)) + dYl[0];
        } else if (wide) {
          slot_reduce<T, NV>(dYl, cpt, lane);
          if (active && storer) dY[(int64_t)ec * g.NY + j0] = (accumulate ? cur.dyo : T(0)) + dYl[0];
        } else {
          for (int off = 1; off < cpt; off <<= 1) {
#pragma unroll
            for (int q = 0; q < NYc; ++q) dYl[q] += __shfl_xor(dYl[q], off);
          }
          if (active && storer) {
            T* dst = dY + (int64_t)ec * g.NY;
#pragma unroll
            for (int q = 0; q < NYc; ++q) dst[q] = accumulate ? dst[q] + dYl[q] : dYl[q];
          }
        }
      });
}

// ------------------------------------------------------------------ dispatch
static TPArgs make_args(const TPLayer& L, int l1, int n_recv, const int* row_ptr, const int* src,
                        const int* pidx) {
  TPArgs a{};
  a.row_ptr = row_ptr;
  a.src = src;
  a.pidx = pidx;
  a.n_recv = n_recv;
  a.Dx = L.xin.width;
  a.P = L.P;
  a.Dm = L.Dm;
  a.NY = L.NY;
  TPDeg& d = a.d;
  const int mul = L.xin.mul[l1];
  d.xoff = L.xin.off[l1];
  d.mul = mul;
  int cpt = 1;
  while (cpt < mul && cpt < kWave) cpt <<= 1;
  d.cpt = cpt;
  d.cpl = (mul + cpt - 1) / cpt;
  d.woff = L.woff[l1];
  for (int p = 0; p < kMaxPathsL1; ++p) {
    d.mo[p] = L.mo[l1][p];
    d.mw[p] = L.mw[l1][p];
  }
  return a;
}

template <typename T, typename S, int L1, int LSH, int LMX, bool SO, int CPT, bool PAIR = false>
static void launch_fwd(const TPArgs& a, const T* Y, const S* x, const S* w, S* M, T inv_k,
                       hipStream_t s) {
  const unsigned grid = (unsigned)((a.n_recv + kRecvPerBlock - 1) / kRecvPerBlock);
  k_tp_fwd<T, S, L1, LSH, LMX, SO, CPT, PAIR>
      <<<grid, kWave * kRecvPerBlock, 0, s>>>(a, Y, x, w, M, inv_k);
}

// Channel pairs (two adjacent channels per lane, one 2-wide access per value) for a degree
// whose 65..128 channels take two per lane anyway, when every row offset is even.
static bool pairable(const TPArgs& a) {
  if (a.d.cpl != 2 || a.d.mul % 2 || a.d.xoff % 2 || a.d.woff % 2 || a.Dx % 2 || a.P % 2 ||
      a.Dm % 2)
    return false;
  for (int p = 0; p < kMaxPathsL1; ++p)
    if (a.d.mo[p] % 2 || a.d.mw[p] % 2) return false;
  return true;
}
template <typename T, typename S, int L1, int LSH, int LMX, bool SO>
static void launch_one(bool fwd, const TPArgs& a, const T* Y, const S* x, const S* w, S* M, T inv_k,
                       const S* G, S* dw, S* dxe, T* dY, int acc, hipStream_t s) {
  // compile-time slot widths for the common channel counts
  // (not in the FP64 form: its paired kernels would need scratch registers)
  constexpr bool kPairs = CPL<L1>::value == 2 && !std::is_same<T, double>::value;
  const bool pair = kPairs && a.d.cpt == 64 && pairable(a);
  if (fwd) {
    if constexpr (kPairs) {
      if (pair) {
        launch_fwd<T, S, L1, LSH, LMX, SO, 64, true>(a, Y, x, w, M, inv_k, s);
        return;
      }
    }
    if (a.d.cpt == 64) launch_fwd<T, S, L1, LSH, LMX, SO, 64>(a, Y, x, w, M, inv_k, s);
    else if (a.d.cpt == 32) launch_fwd<T, S, L1, LSH, LMX, SO, 32>(a, Y, x, w, M, inv_k, s);
    else launch_fwd<T, S, L1, LSH, LMX, SO, 0>(a, Y, x, w, M, inv_k, s);
    return;
  }
  const unsigned grid =
      (unsigned)((((int64_t)a.n_recv << a.split_log) + kRecvPerBlock - 1) / kRecvPerBlock);
  const unsigned block = kWave * kRecvPerBlock;
#define SN_TP_BWD(DX, CPT) \
  k_tp_bwd<T, S, L1, LSH, LMX, SO, DX, CPT><<<grid, block, 0, s>>>(a, Y, x, w, G, dw, dxe, dY, acc)
  if constexpr (kPairs) {
    if (pair) {
      if (dxe)
        k_tp_bwd<T, S, L1, LSH, LMX, SO, true, 64, true>
            <<<grid, block, 0, s>>>(a, Y, x, w, G, dw, dxe, dY, acc);
      else
        k_tp_bwd<T, S, L1, LSH, LMX, SO, false, 64, true>
            <<<grid, block, 0, s>>>(a, Y, x, w, G, dw, dxe, dY, acc);
      return;
    }
  }
  if (dxe) {
    if (a.d.cpt == 64) SN_TP_BWD(true, 64);
    else if (a.d.cpt == 32) SN_TP_BWD(true, 32);
    else SN_TP_BWD(true, 0);
  } else {
    if (a.d.cpt == 64) SN_TP_BWD(false, 64);
    else if (a.d.cpt == 32) SN_TP_BWD(false, 32);
    else SN_TP_BWD(false, 0);
  }
#undef SN_TP_BWD
}

template <typename T, typename S>
static void run(const TPLayer& L, bool fwd, int n_recv, const int* row_ptr, const int* src,
                const int* pidx, const T* Y, const S* x, const S* w, S* M, T inv_k, const S* G,
                S* dw, S* dxe, T* dY, bool accumulate, hipStream_t s) {
  if (n_recv <= 0) return;
  bool first = true;
  for (int l1 = 0; l1 <= L.lmax; ++l1) {
    if (L.xin.mul[l1] == 0) continue;
    TPArgs a = make_args(L, l1, n_recv, row_ptr, src, pidx);
    if (!fwd) a.split_log = tp_split_log(n_recv);
    const int acc = (accumulate || !first) ? 1 : 0;
    first = false;
#define SN_TP_CASE(LL1, LSH, LMX, SO)                                                        \
  if (l1 == LL1 && L.lsh == LSH && L.lmax == LMX && L.scalar_only == SO) {                   \
    launch_one<T, S, LL1, LSH, LMX, SO>(fwd, a, Y, x, w, M, inv_k, G, dw, dxe, dY, acc, s);     \
    continue;                                                                                \
  }
    SN_TP_CASE(0, 1, 1, false) SN_TP_CASE(1, 1, 1, false)
    SN_TP_CASE(0, 1, 1, true) SN_TP_CASE(1, 1, 1, true)
    SN_TP_CASE(0, 2, 2, false) SN_TP_CASE(1, 2, 2, false) SN_TP_CASE(2, 2, 2, false)
    SN_TP_CASE(0, 2, 2, true) SN_TP_CASE(1, 2, 2, true) SN_TP_CASE(2, 2, 2, true)
    SN_TP_CASE(0, 3, 3, false) SN_TP_CASE(1, 3, 3, false) SN_TP_CASE(2, 3, 3, false)
    SN_TP_CASE(3, 3, 3, false)
    SN_TP_CASE(0, 3, 3, true) SN_TP_CASE(1, 3, 3, true) SN_TP_CASE(2, 3, 3, true)
    SN_TP_CASE(3, 3, 3, true)
#undef SN_TP_CASE
    throw std::invalid_argument("no tensor-product kernel for this degree combination");
  }
}

template <typename T, typename S>
void launch_tp_fwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src,
                   const int* pidx, const T* Y, const S* x, const S* w, S* M, T inv_k,
                   hipStream_t s) {
  run<T, S>(L, true, n_recv, row_ptr, src, pidx, Y, x, w, M, inv_k, nullptr, nullptr, nullptr,
            nullptr, false, s);
}
template <typename T, typename S>
void launch_tp_bwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src,
                   const int* pidx, const T* Y, const S* x, const S* w, const S* G, S* dw, S* dxe,
                   T* dY, bool accumulate, hipStream_t s) {
  run<T, S>(L, false, n_recv, row_ptr, src, pidx, Y, x, w, nullptr, T(0), G, dw, dxe, dY,
            accumulate, s);
}

#define SN_TP_INST(T, S)                                                                       \
  template void launch_tp_fwd<T, S>(const TPLayer&, int, const int*, const int*, const int*,     \
                                    const T*, const S*, const S*, S*, T, hipStream_t);          \
  template void launch_tp_bwd<T, S>(const TPLayer&, int, const int*, const int*, const int*,     \
                                    const T*, const S*, const S*, const S*, S*, S*, T*, bool,    \
                                    hipStream_t);

}  // namespace sn
