// Host-side launchers of the libsn kernels (one declaration per kernel family).
#pragma once

#include "common.h"

namespace sn {

// ---------------------------------------------------------------- graph build
struct BinGrid {
  int nb[3];        // bins per axis over the extended fractional region
  double bw[3];     // bin width (fractional units), >= delta
  double delta[3];  // shell half-width (fractional units) = (r_c + skin) / perpendicular width
  int nimg[3];      // image-shift search range per axis
  double lo[3], hi[3];  // the region's own fractional box [lo, hi); bins cover [lo-delta, hi+delta)
};

// exclusive scan of n ints into out[0..n] (out[n] = total); tmp needs scan_tmp_ints(n) ints
size_t scan_tmp_ints(int64_t n);
void scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t s);

// Geometry of one region of a packed graph.  A region is one spatial subdomain of a
// structure (the whole cell unless the structure is split into ndom[0] x ndom[1] x ndom[2]
// fractional boxes).  Each region has its own ghost shell; edges never cross regions.
struct StructParams {
  double H[9], Hinv[9];  // cell (rows a1 a2 a3) and its inverse
  BinGrid g;
  int bin_base;          // first global bin key of this region
  int first_region;      // index of the structure's first region (its regions are consecutive)
  int ndom[3];           // the structure's subdomain grid
  int pad;
};

// sid: first region of each atom's structure; rid receives the atom's own region.
void launch_wrap_bin(int n, const double* pos, const int* sid, const StructParams* sp, double* posw,
                     double* frac, int* key, int* rid, int* err, hipStream_t s);
void launch_count_keys(int n, const int* key, int* count, hipStream_t s);
void launch_scatter_keys(int n, const int* key, const int* start, int* cursor, int* items,
                         hipStream_t s);
void launch_sort_segments(int nseg, const int* start, int* items, hipStream_t s);
void launch_gather_local(int n, const int* order, const double* posw, const double* frac,
                         const int* spec_orig, const int* sid_orig, double* pos_ext,
                         double* frac_ext, int* spec_ext, int* sid_ext, hipStream_t s);
void launch_ghost_count(int n, const double* frac, const int* sid, const StructParams* sp,
                        int* count, hipStream_t s);
// sid: structure id per extended row (locals on input; ghost rows filled here)
void launch_ghost_fill(int n, const double* frac, const double* pos, const int* spec, int* sid,
                       const StructParams* sp, const int* gptr, int* owner, int* shift,
                       double* pos_ext, double* frac_ext, int* spec_ext, hipStream_t s);
void launch_bin_keys(int n, const double* frac, const int* sid, const StructParams* sp, int* key,
                     hipStream_t s);
void launch_edge_count(int n, const double* pos_ext, const double* frac_ext, const int* sid,
                       const StructParams* sp, const int* cell_start, const int* cell_items,
                       double rc2, int* count, int* err, hipStream_t s);
void launch_edge_fill(int n, const double* pos_ext, const double* frac_ext, const int* sid,
                      const StructParams* sp, const int* cell_start, const int* cell_items,
                      double rc2, const int* row_ptr, int* src, int* recv, hipStream_t s);

// Compaction of a list built out to r_c + skin to the pairs now inside r_c (both edges of a
// pair kept or dropped together; order preserved), for evaluating a kept list: the edge
// arrays, the pair table, the receiver and sender offsets and the per-structure edge
// offsets are rewritten into `CompactOut`.  The compacted counts are escan[E] (edges) and
// pscan[np] (pairs).  Scratch arrays hold np + 1 (active, pscan) or E + 1 ints; tmp
// scan_tmp_ints(max(E, np) + 1).
struct CompactIn {
  int64_t E, np;
  int n_local, n_ext, n_struct;
  const int *row_ptr, *src, *recv, *pidx, *pe1, *pe2, *send_ptr, *send_idx, *edge_off;
  const double* pos_ext;
  double r_cut;
};
struct CompactOut {
  int *row_ptr, *src, *recv, *pidx, *pe1, *pe2, *send_ptr, *send_idx, *edge_off;
};
struct CompactScratch {
  int *active, *pscan, *keep, *escan, *keep_s, *sscan, *tmp;
};
void launch_compact_active(const CompactIn& in, const CompactOut& out, CompactScratch& t,
                           hipStream_t s);

// Reverse-edge map and undirected pairs: rev[e] (-1 if none), pidx[e] (pair of each edge),
// pe1[p] (canonical edge of pair p, the lower id) and pe2[p] (its reverse or -1).  The
// number of pairs is fscan[E].  tmp is scan scratch.
void launch_pairs(int64_t E, int n_local, const int* recv, const int* src, const int* row_ptr,
                  const int* owner, const int* shift, int* rev, int* flag, int* fscan, int* tmp,
                  int* pidx, int* pe1, int* pe2, hipStream_t s);

// ---------------------------------------------------------------- edge basis
template <typename T>
void launch_edge_basis(int64_t E, const int* recv, const int* src, const double* pos_ext,
                       double r_cut, int n_basis, int p, int l_sh, T* Y, T* rho, hipStream_t s);
template <typename T>
void launch_edge_grad(int64_t E, const int* recv, const int* src, const double* pos_ext,
                      double r_cut, int n_basis, int p, int l_sh, const T* dY, const T* drho,
                      double* g, hipStream_t s);

// ---------------------------------------------------------------- dense algebra
// C[M x N] (=|+=) alpha * A[M x K] * op(B); op(B) = B (K x N, ld ldb) or B^T (B is N x K).
// Operands of types TA/TB are accumulated in TACC and stored as TC; with bf16_operands
// both operands are first rounded to bfloat16 (round-to-nearest-even).
template <typename TA, typename TB, typename TC, typename TACC>
void launch_gemm(int64_t M, int N, int K, const TA* A, RowMap am, const TB* B, int ldb, bool bt,
                 TC* C, RowMap cm, TACC alpha, bool accumulate, bool bf16_operands, hipStream_t s);

// Same contraction on the matrix cores with float32 accumulation (bfloat16 operands
// when bf16 is set).
template <typename TA, typename TB, typename TC>
void launch_gemm_mfma(int64_t M, int N, int K, const TA* A, RowMap am, const TB* B, int ldb, bool bt,
                      TC* C, RowMap cm, float alpha, bool accumulate, bool bf16, hipStream_t s);

// Several independent contractions of the same operand types and B layout in one launch
// (the per-degree blocks of one channel-mixing layer): every problem's tiles are spread
// over the grid together.  Each problem is computed exactly as by the single launches.
template <typename TA, typename TB, typename TC>
struct GemmDesc {
  int64_t M;
  int N, K;
  const TA* A;
  RowMap am;
  const TB* B;
  int ldb;
  TC* C;
  RowMap cm;
  double alpha;
  int accumulate;
};
constexpr int kMaxGemmGroup = 4;
constexpr int64_t kGroupMaxTiles = 1024;  // larger groups launch problem by problem
template <typename TA, typename TB, typename TC, typename TACC>
void launch_gemm_group(int n, const GemmDesc<TA, TB, TC>* d, bool bt, bool bf16_operands,
                       hipStream_t s);
template <typename TA, typename TB, typename TC>
void launch_gemm_mfma_group(int n, const GemmDesc<TA, TB, TC>* d, bool bt, bool bf16, hipStream_t s);

// Vector-unit radial-MLP hidden layers over pairs (float64 form): rows of rho and drho
// are taken at rows[p].
template <typename T>
void launch_mlp_hidden_fwd(int64_t np, const int* rows, const T* rho, int nb, int hidden,
                           const T* Wa, const T* Wb, T c, T* z2, hipStream_t s);
// With z1, da1, da2 (may be null): also the per-pair hidden activation and pre-activation
// gradients [np x hidden] for the weight gradients.
template <typename T>
void launch_mlp_hidden_bwd(int64_t np, const int* rows, const T* rho, int nb, int hidden,
                           const T* Wa, const T* Wb, T c, const T* dz2, T* drho, bool accumulate,
                           hipStream_t s, T* z1 = nullptr, T* da1 = nullptr, T* da2 = nullptr);
// out[p] = dw[2p] + dw[2p+1] (second term absent when pe2[p] < 0), rows of width P, stored
// type S widened to T
template <typename S, typename T>
void launch_pair_sum(int64_t np, const int* pe1, const int* pe2, const S* dw, int P, T* out,
                     hipStream_t s);

// ---------------------------------------------------------------- training (weight gradients)
// dW[k][n] = scale * sum_r A[r'][k] B[r][n] over `rows` rows, float64 accumulation, fixed
// chunk order: r' = aidx[r] when aidx is given (else r); with onehot, A[r'][k] = (onehot[r'] == k).
// partial needs wgrad_chunks(rows) * K * N doubles.
int64_t wgrad_chunks(int64_t rows);
template <typename TA, typename TB>
void launch_wgrad(int64_t rows, int K, int N, const TA* A, RowMap am, const int* aidx,
                  const int* onehot, const TB* B, RowMap bm, double scale, double* partial,
                  double* out, hipStream_t s);
void launch_atom_grad(int n, const int* region, int regions_per_struct, const double* grad,
                      double* g_atom, hipStream_t s);
template <typename H>
void launch_seed_rows(int n, const double* v, int C0, double sigma, const double* g_atom, H* dh,
                      int ldh, hipStream_t s);
void launch_readout_wgrad(int C0, const double* u, const double* wr1, const double* wr2,
                          double sigma, double* g_wr1, double* g_wr2, hipStream_t s);
// out_i = pos_i + eps (v_i + U_b pos_i) with b = atom_struct[i] and U[b] row-major 3 x 3
void launch_perturb(int64_t n, const double* pos, const double* v, const double* U,
                    const int* atom_struct, double eps, double* out, hipStream_t s);
void launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s);
void launch_fill_f64(int64_t n, double v, double* y, hipStream_t s);

// Fused radial MLP (hidden layers + output layer) on the matrix cores, over undirected
// pairs: pair p takes rho of edge pe1[p]; the backward sums the pair-major dE/dw rows 2p
// and 2p+1 (the latter absent when pe2[p] < 0) and adds drho into row pe1[p].  P must be
// a multiple of 8.  The output weights Wc [64 x P] come as 64-column panels, each 64 x 64
// contiguous and zero past column P (see wc_panels).
// BF16 form: bfloat16 operands for the two P-wide contractions and bfloat16 storage of w
// and dE/dw; Wcp is [panel][c][j] for the forward, [panel][j][c] for the backward.
void launch_mlp_fused_fwd(int64_t np, const int* pe1, const float* rho, const float* Wa,
                          const float* Wb, const bf16_t* Wcp, int P, float c, bf16_t* w,
                          hipStream_t s);
void launch_mlp_fused_bwd(int64_t np, const int* pe1, const int* pe2, const float* rho,
                          const float* Wa, const float* Wb, const bf16_t* Wcp, int P, float c,
                          const bf16_t* dw, float* drho, bool accumulate, hipStream_t s);
// FP32 form: float32 storage, the P-wide contractions in three-part bfloat16 arithmetic
// (float32-level results).  Wc3 holds per panel the three bfloat16 parts x0, x1, x2 of
// every weight (x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1)): each [c][j] for
// the forward, each [j][c] for the backward.
void launch_mlp_fused_fwd_split(int64_t np, const int* pe1, const float* rho, const float* Wa,
                                const float* Wb, const bf16_t* Wc3, int P, float c, float* w,
                                hipStream_t s);
void launch_mlp_fused_bwd_split(int64_t np, const int* pe1, const int* pe2, const float* rho,
                                const float* Wa, const float* Wb, const bf16_t* Wc3, int P, float c,
                                const float* dw, float* drho, bool accumulate, hipStream_t s);

// ---------------------------------------------------------------- tensor product
struct TPTask {  // one wave's work: one degree l1, 64 lanes over channels x edges
  int l1;
  int u0;        // first channel
  int cpt;       // channels per edge slot (power of two <= 64)
};

constexpr int kMaxPathsL1 = 16;  // paths per input degree (11 at most for l <= 3)

struct TPLayer {
  int lmax, lsh;
  bool scalar_only;     // last block: only l3 = 0 paths
  IrrepLayout xin;      // layout of the sender feature rows
  int P;                // radial weights per edge
  int woff[kNumL];      // first weight of the paths with each l1
  int Dm;               // mid (message) row width
  // per l1, per local path index: offset of (l3 block + channel start) in M, and l3 mid width
  int mo[kNumL][kMaxPathsL1];
  int mw[kNumL][kMaxPathsL1];
  int n_tasks;
  TPTask tasks[16];
  int NY;               // (l_sh + 1)^2
};

// Messages M [n_recv x Dm] of one block; w is indexed by the edge's pair pidx[e] / 2.
// S is the storage type of x, w, M, dE/dM, dE/dw and the per-edge dE/dx rows (T, or bf16_t
// in the bfloat16 form); arithmetic is in T.
template <typename T, typename S>
void launch_tp_fwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src,
                   const int* pidx, const T* Y, const S* x, const S* w, S* M, T inv_k,
                   hipStream_t s);
// The adjoint of a small graph runs 2^tp_split_log(n_recv) waves per receiver, each over a
// contiguous slice of its edges (until about 2,048 waves run; at most 8 per receiver).
// Every edge's adjoint outputs are computed whole by one wave, so results do not depend on
// the split.  (The forward is not split: partial message sums would make a structure's
// result depend on the size of the packed graph it is evaluated in.)
constexpr int kTPSplitWaves = 2048;
inline int tp_split_log(int n_recv) {
  int k = 0;
  while (n_recv > 0 && ((int64_t)n_recv << k) < kTPSplitWaves && k < 3) ++k;
  return k;
}
// Adjoint: writes dE/dw [E x P], per-edge dE/dx_sender rows dxe [E x Dx] (skipped when dxe is
// null), and dE/dY [E x NY] (added to the existing values when accumulate is set).
template <typename T, typename S>
void launch_tp_bwd(const TPLayer& L, int n_recv, const int* row_ptr, const int* src,
                   const int* pidx, const T* Y, const S* x, const S* w, const S* G, S* dw,
                   S* dxe, T* dY, bool accumulate, hipStream_t s);

// ---------------------------------------------------------------- node-level and reductions
template <typename T>
void launch_embed(int rows, const int* spec, const T* Wemb, int C0, T* h, int ldh, hipStream_t s);
template <typename T>
void launch_ghost_refresh(int n_local, int n_ghost, const int* owner, T* x, int width,
                          hipStream_t s);
template <typename T>
void launch_gate_fwd(int n, bool last, IrrepLayout yl, IrrepLayout hl, const T* y, T* h, T c,
                     hipStream_t s);
template <typename TY, typename TG>
void launch_gate_bwd(int n, bool last, IrrepLayout yl, IrrepLayout hl, const TY* y, const TG* dh,
                     TG* dy, TY c, hipStream_t s);
template <typename T>
void launch_readout(int n, const T* h, int ldh, const double* v, int C0, double sigma,
                    const double* shift, const int* spec, double* atom_e, hipStream_t s);
template <typename T>
void launch_fill_rows(int n, const double* v, int C0, double scale, T* dh, int ldh,
                      hipStream_t s);
template <typename T, typename H>
void launch_sender_reduce(int n_rows, const int* sptr, const int* sidx, const T* dxe, int width,
                          H* dx, hipStream_t s);
template <typename T>
void launch_ghost_fold(int n_local, const int* gptr, const T* dx_ext, T* dx, int width,
                       hipStream_t s);
template <typename T>
void launch_dY_reduce(int64_t E, int n_tasks, int NY, const T* part, T* dY, bool accumulate,
                      hipStream_t s);
void launch_forces(int n_local, const int* row_ptr, const int* sptr, const int* sidx,
                   const int* gptr, const double* g, double* F, hipStream_t s);
// Per-structure sums: chunks holds (structure, begin, end) triples; first[b]..first[b+1]
// are structure b's chunks.  Energy sums atom energies; virial sums -d_e (x) g_e over edges.
void launch_seg_energy(int nchunks, const int* chunks, const double* atom_e, double* partial,
                       hipStream_t s);
void launch_seg_virial(int nchunks, const int* chunks, const int* recv, const int* src,
                       const double* pos_ext, const double* g, double* partial, hipStream_t s);
// gscale: per-structure factors in device memory (null: 1)
void launch_seg_finalize(int B, const int* first, const double* partial, int width, double* out,
                         const double* gscale, hipStream_t s);
void launch_unpermute(int n, const int* order, const double* in_rows, int width,
                      double* out_rows, const double* gscale, const int* sid_orig,
                      int regions_per_struct, hipStream_t s);

// Kept graph, moved atoms: local rows from pos[order[k]] + wrap_off[k], ghost rows from
// owner row + shift . H.  wrap_off is recorded at build time by launch_wrap_offsets.
void launch_refresh_positions(int n, int n_ghost, const int* order, const double* pos,
                              const double* wrap_off, const int* owner, const int* shift,
                              const int* sid_ext, const StructParams* sp, double* pos_ext,
                              hipStream_t s);
void launch_wrap_offsets(int n, const int* order, const double* pos, const double* pos_ext,
                         double* wrap_off, hipStream_t s);
// Velocity-Verlet half step (stage 0: kick + drift, stage 1: kick); a = F * inv_mass.
void launch_verlet(int n, double* pos, double* vel, const double* F, const double* inv_mass,
                   double dt, int stage, hipStream_t s);
// Block-partial scratch (doubles) needed by the two kernels below for n atoms.
int md_partials(int n);
// Nose-Hoover half-step operator on vel (n x 3); state = {xi, eta, scale, K} in device memory;
// gkT = degrees of freedom x kT (eV), Q the thermostat mass (eV fs^2).
void launch_nh_half(int n, double* vel, const double* inv_mass, double dt, double gkT, double Q,
                    double* state, double* part, hipStream_t s);
// out[0] = max_i |pos_i - ref_i|^2 (device).
void launch_max_disp2(int n, const double* pos, const double* ref, double* part, double* out,
                      hipStream_t s);



}  // namespace sn
