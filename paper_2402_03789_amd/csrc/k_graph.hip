// Graph build: wrap, cell binning, ghost shell, receiver and sender CSR.
//
// Subdomains with ghost shells (paper section 3.1): a structure is one subdomain (its
// whole cell) or a grid of fractional boxes.  Every image of an atom whose fractional
// coordinates fall within (r_c + skin) / w_a of a subdomain's box on each axis (w_a:
// perpendicular width), other than the atom itself in its own subdomain, is a ghost of that
// subdomain with an owner and an integer image shift.  Edges join a local receiver to any local or
// ghost sender closer than r_c (section 2), found by scanning the 27 bins
// around the receiver on a grid over the extended fractional region whose
// bin width is at least the shell half-width.  Every list is made
// deterministic: bins are filled and then sorted by point index, edges are
// emitted in bin-scan order, and sender segments are sorted by edge id.
#include "kernels.h"

#include <climits>

namespace sn {

// ------------------------------------------------------------------ exclusive scan
constexpr int kScanBlock = 1024;

__global__ void k_scan_block(const int* __restrict__ in, int* __restrict__ out, int64_t n,
                             int* __restrict__ block_sums) {
  __shared__ int s[kScanBlock];
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int v = (i < n) ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;  // exclusive
  if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int* __restrict__ out, int64_t n, const int* __restrict__ offs) {
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += offs[blockIdx.x];
}

__global__ void k_scan_total(const int* __restrict__ in, int* __restrict__ out, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = (n > 0 ? out[n - 1] + in[n - 1] : 0);
}

size_t scan_tmp_ints(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (true) {
    int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    total += 2 * nb + 1;
    if (nb <= 1) break;
    m = nb;
  }
  return total + 16;
}

void scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t s) {
  if (n <= 0) {
    k_scan_total<<<1, 1, 0, s>>>(in, out, 0);
    return;
  }
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int* sums = tmp;
  k_scan_block<<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, n, sums);
  if (nb > 1) {
    int* sums_scan = tmp + nb;
    scan_exclusive(sums, sums_scan, nb, tmp + 2 * nb + 1, s);
    k_scan_add<<<(unsigned)nb, kScanBlock, 0, s>>>(out, n, sums_scan);
  }
  k_scan_total<<<1, 1, 0, s>>>(in, out, n);
}

// ------------------------------------------------------------------ binning helpers
// Several structures can share one packed graph: every point carries its structure id,
// and structure b bins into the global key range [bin_base, bin_base + nb0*nb1*nb2).
__device__ inline int bin_axis(double f, const BinGrid& g, int a) {
  int b = (int)floor((f - g.lo[a] + g.delta[a]) / g.bw[a]);
  return min(max(b, 0), g.nb[a] - 1);
}
// subdomain index of fractional coordinate f on an axis split into n boxes [j/n, (j+1)/n)
__device__ inline int dom_axis(double f, int n) {
  int j = min(max((int)floor(f * n), 0), n - 1);
  if (j > 0 && f < (double)j / n) --j;
  if (j < n - 1 && f >= (double)(j + 1) / n) ++j;
  return j;
}
__device__ inline int bin_lin(const double* f, const BinGrid& g) {
  return (bin_axis(f[0], g, 0) * g.nb[1] + bin_axis(f[1], g, 1)) * g.nb[2] + bin_axis(f[2], g, 2);
}

__global__ void k_wrap_bin(int n, const double* __restrict__ pos, const int* __restrict__ sid,
                           const StructParams* __restrict__ sp, double* __restrict__ posw,
                           double* __restrict__ frac, int* __restrict__ key, int* __restrict__ rid,
                           int* __restrict__ err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const StructParams& P0 = sp[sid[i]];
  double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) {
    atomicOr(err, 1);
    p[0] = p[1] = p[2] = 0.0;
  }
  double f[3];
  for (int a = 0; a < 3; ++a) {
    // row vector p times Hinv
    double v = p[0] * P0.Hinv[0 * 3 + a] + p[1] * P0.Hinv[1 * 3 + a] + p[2] * P0.Hinv[2 * 3 + a];
    v -= floor(v);
    if (v >= 1.0) v = 0.0;
    f[a] = v;
  }
  for (int a = 0; a < 3; ++a) {
    frac[3 * i + a] = f[a];
    posw[3 * i + a] = f[0] * P0.H[0 * 3 + a] + f[1] * P0.H[1 * 3 + a] + f[2] * P0.H[2 * 3 + a];
  }
  // the atom's subdomain (region) within its structure
  const int r = sid[i] + (dom_axis(f[0], P0.ndom[0]) * P0.ndom[1] + dom_axis(f[1], P0.ndom[1])) *
                             P0.ndom[2] +
                dom_axis(f[2], P0.ndom[2]);
  rid[i] = r;
  key[i] = sp[r].bin_base + bin_lin(f, sp[r].g);
}

__global__ void k_count_keys(int n, const int* __restrict__ key, int* __restrict__ count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&count[key[i]], 1);
}

__global__ void k_scatter_keys(int n, const int* __restrict__ key, const int* __restrict__ start,
                               int* __restrict__ cursor, int* __restrict__ items) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = key[i];
  int pos = start[k] + atomicAdd(&cursor[k], 1);
  items[pos] = i;
}

// Ascending sort of each segment (bin or sender lists: distinct item indices), one wave
// per segment: every value's final position is the number of smaller values in the
// segment (counted through cross-lane broadcasts), so each lane places its values
// directly.  Segments of up to 64 * kSortChunks items; longer ones (none in practice)
// fall back to an insertion sort by one lane.
constexpr int kSortChunks = 8;
__global__ __launch_bounds__(256) void k_sort_segments(int nseg, const int* __restrict__ start,
                                                       int* __restrict__ items) {
  const int sg = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (sg >= nseg) return;
  const int lane = threadIdx.x & 63;
  const int a = start[sg], n = start[sg + 1] - a;
  if (n <= 1) return;
  if (n > 64 * kSortChunks) {
    if (lane == 0) {
      for (int i = a + 1; i < a + n; ++i) {
        const int v = items[i];
        int j = i - 1;
        while (j >= a && items[j] > v) {
          items[j + 1] = items[j];
          --j;
        }
        items[j + 1] = v;
      }
    }
    return;
  }
  const int nc = (n + 63) >> 6;
  int v[kSortChunks], rank[kSortChunks];
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    const int i = 64 * c + lane;
    v[c] = (c < nc && i < n) ? items[a + i] : INT_MAX;
    rank[c] = 0;
  }
#pragma unroll
  for (int cs = 0; cs < kSortChunks; ++cs) {
    if (cs >= nc) break;
    const int m = min(64, n - 64 * cs);
    for (int j = 0; j < m; ++j) {
      const int w = __shfl(v[cs], j);
#pragma unroll
      for (int c = 0; c < kSortChunks; ++c) rank[c] += w < v[c] ? 1 : 0;
    }
  }
#pragma unroll
  for (int c = 0; c < kSortChunks; ++c) {
    const int i = 64 * c + lane;
    if (c < nc && i < n) items[a + rank[c]] = v[c];
  }
}

__global__ void k_gather_local(int n, const int* __restrict__ order, const double* __restrict__ posw,
                               const double* __restrict__ frac, const int* __restrict__ spec_orig,
                               const int* __restrict__ sid_orig, double* __restrict__ pos_ext,
                               double* __restrict__ frac_ext, int* __restrict__ spec_ext,
                               int* __restrict__ sid_ext) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int o = order[k];
  for (int a = 0; a < 3; ++a) {
    pos_ext[3 * k + a] = posw[3 * o + a];
    frac_ext[3 * k + a] = frac[3 * o + a];
  }
  spec_ext[k] = spec_orig[o];
  sid_ext[k] = sid_orig[o];
}

__device__ inline bool in_shell(const double* f, int sx, int sy, int sz, const BinGrid& g) {
  double v[3] = {f[0] + sx, f[1] + sy, f[2] + sz};
  for (int a = 0; a < 3; ++a)
    if (!(v[a] >= g.lo[a] - g.delta[a] && v[a] < g.hi[a] + g.delta[a])) return false;
  return true;
}

// Ghosts of local atom k: every image (shift n) inside the extended box of a region of
// its structure, except the atom itself in its own region (n = 0).  With one region per
// structure these are the periodic images around the cell; with several, an atom is also
// a shift-0 ghost of every neighbouring subdomain whose shell reaches it.  Order: region,
// then shift (owner-major overall, so each owner's ghosts are contiguous).
template <class F>
__device__ inline void for_each_ghost(const double* f, int own_region,
                                      const StructParams* __restrict__ sp, F&& emit) {
  const StructParams& P = sp[own_region];
  const int nreg = P.ndom[0] * P.ndom[1] * P.ndom[2];
  const int first = P.first_region;
  const int ni[3] = {P.g.nimg[0], P.g.nimg[1], P.g.nimg[2]};
  for (int d = first; d < first + nreg; ++d) {
    const BinGrid g = sp[d].g;  // one copy in registers for the image loop
    for (int sx = -ni[0]; sx <= ni[0]; ++sx)
      for (int sy = -ni[1]; sy <= ni[1]; ++sy)
        for (int sz = -ni[2]; sz <= ni[2]; ++sz) {
          if (sx == 0 && sy == 0 && sz == 0 && d == own_region) continue;
          if (in_shell(f, sx, sy, sz, g)) emit(d, sx, sy, sz);
        }
  }
}

__global__ void k_ghost_count(int n, const double* __restrict__ frac, const int* __restrict__ sid,
                              const StructParams* __restrict__ sp, int* __restrict__ count) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double f[3] = {frac[3 * k], frac[3 * k + 1], frac[3 * k + 2]};
  int c = 0;
  for_each_ghost(f, sid[k], sp, [&](int, int, int, int) { ++c; });
  count[k] = c;
}

__global__ void k_ghost_fill(int n, const double* __restrict__ frac, const double* __restrict__ pos,
                             const int* __restrict__ spec, int* __restrict__ sid,
                             const StructParams* __restrict__ sp, const int* __restrict__ gptr,
                             int* __restrict__ owner, int* __restrict__ shift,
                             double* __restrict__ pos_ext, double* __restrict__ frac_ext,
                             int* __restrict__ spec_ext) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const StructParams& P = sp[sid[k]];
  double f[3] = {frac[3 * k], frac[3 * k + 1], frac[3 * k + 2]};
  int w = gptr[k];
  for_each_ghost(f, sid[k], sp, [&](int d, int sx, int sy, int sz) {
    owner[w] = k;
    shift[3 * w] = sx;
    shift[3 * w + 1] = sy;
    shift[3 * w + 2] = sz;
    const int r = n + w;
    for (int a = 0; a < 3; ++a)
      pos_ext[3 * r + a] =
          pos[3 * k + a] + sx * P.H[0 * 3 + a] + sy * P.H[1 * 3 + a] + sz * P.H[2 * 3 + a];
    frac_ext[3 * r] = f[0] + sx;
    frac_ext[3 * r + 1] = f[1] + sy;
    frac_ext[3 * r + 2] = f[2] + sz;
    spec_ext[r] = spec[k];
    sid[r] = d;
    ++w;
  });
}

__global__ void k_bin_keys(int n, const double* __restrict__ frac, const int* __restrict__ sid,
                           const StructParams* __restrict__ sp, int* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const StructParams& P = sp[sid[i]];
  double f[3] = {frac[3 * i], frac[3 * i + 1], frac[3 * i + 2]};
  key[i] = P.bin_base + bin_lin(f, P.g);
}

// Edges of receiver k: every extended point s != k of the 27 bins around k's bin with
// |r_s - r_k|^2 < rc2, in bin order (x, then y, then z) and item order within a bin.  One
// wave per receiver: lanes 0..26 take one neighbouring bin each, a wave prefix sum lays
// the bins' items out as one candidate list, and the lanes test 64 candidates at a time;
// hits are numbered by a ballot prefix, so the edge order is the same as a serial scan.
template <bool FILL>
__global__ __launch_bounds__(256) void k_edges(int n, const double* __restrict__ pos_ext,
                                               const double* __restrict__ frac_ext,
                                               const int* __restrict__ sid,
                                               const StructParams* __restrict__ sp,
                                               const int* __restrict__ cell_start,
                                               const int* __restrict__ cell_items, double rc2,
                                               int* __restrict__ count, int* __restrict__ err,
                                               const int* __restrict__ row_ptr,
                                               int* __restrict__ src, int* __restrict__ recv) {
  const int k = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (k >= n) return;
  const int lane = threadIdx.x & 63;
  const StructParams& P = sp[sid[k]];
  const BinGrid g = P.g;
  const double p0 = pos_ext[3 * k], p1 = pos_ext[3 * k + 1], p2 = pos_ext[3 * k + 2];
  int b[3];
  for (int a = 0; a < 3; ++a) b[a] = bin_axis(frac_ext[3 * k + a], g, a);
  // this lane's bin (lanes 0..26): offsets (dx, dy, dz) in lexicographic order
  int c0 = 0, cn = 0;
  if (lane < 27) {
    const int bx = b[0] + lane / 9 - 1, by = b[1] + (lane / 3) % 3 - 1, bz = b[2] + lane % 3 - 1;
    if (bx >= 0 && bx < g.nb[0] && by >= 0 && by < g.nb[1] && bz >= 0 && bz < g.nb[2]) {
      const int cell = P.bin_base + (bx * g.nb[1] + by) * g.nb[2] + bz;
      c0 = cell_start[cell];
      cn = cell_start[cell + 1] - c0;
    }
  }
  int incl = cn;  // inclusive prefix of the bin sizes over lanes
  for (int o = 1; o < 32; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const int total = __shfl(incl, 26);
  int w = FILL ? row_ptr[k] : 0;
  int c = 0;
  for (int v0 = 0; v0 < total; v0 += 64) {
    const int v = v0 + lane;
    const int vc = min(v, total - 1);  // every lane takes part in the cross-lane reads
    int j = 0;                          // first bin whose inclusive prefix exceeds vc
    for (int step = 16; step > 0; step >>= 1) {
      const int t = __shfl(incl, j + step - 1);
      if (j + step - 1 < 27 && t <= vc) j += step;
    }
    const int first = __shfl(incl, j) - __shfl(cn, j);
    const int q = __shfl(c0, j) + (vc - first);
    bool hit = false;
    int s = 0;
    if (v < total) {
      s = cell_items[q];
      if (s != k) {
        const double dx = pos_ext[3 * s] - p0, dy = pos_ext[3 * s + 1] - p1,
                     dz = pos_ext[3 * s + 2] - p2;
        const double r2 = dx * dx + dy * dy + dz * dz;
        hit = r2 < rc2;
        if (!FILL && hit && r2 < 1e-16) atomicOr(err, 2);
      }
    }
    const unsigned long long m = __ballot(hit);
    if (FILL) {
      if (hit) {
        const int at = w + __popcll(m & ((1ull << lane) - 1ull));
        src[at] = s;
        recv[at] = k;
      }
      w += __popcll(m);
    } else {
      c += __popcll(m);
    }
  }
  if (!FILL && lane == 0) count[k] = c;
}

// ------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_wrap_bin(int n, const double* pos, const int* sid, const StructParams* sp, double* posw,
                     double* frac, int* key, int* rid, int* err, hipStream_t s) {
  if (n > 0) k_wrap_bin<<<nblk(n, 256), 256, 0, s>>>(n, pos, sid, sp, posw, frac, key, rid, err);
}
void launch_count_keys(int n, const int* key, int* count, hipStream_t s) {
  if (n > 0) k_count_keys<<<nblk(n, 256), 256, 0, s>>>(n, key, count);
}
void launch_scatter_keys(int n, const int* key, const int* start, int* cursor, int* items,
                         hipStream_t s) {
  if (n > 0) k_scatter_keys<<<nblk(n, 256), 256, 0, s>>>(n, key, start, cursor, items);
}
void launch_sort_segments(int nseg, const int* start, int* items, hipStream_t s) {
  if (nseg > 0) k_sort_segments<<<nblk(nseg, 4), 256, 0, s>>>(nseg, start, items);
}
void launch_gather_local(int n, const int* order, const double* posw, const double* frac,
                         const int* spec_orig, const int* sid_orig, double* pos_ext,
                         double* frac_ext, int* spec_ext, int* sid_ext, hipStream_t s) {
  if (n > 0)
    k_gather_local<<<nblk(n, 256), 256, 0, s>>>(n, order, posw, frac, spec_orig, sid_orig, pos_ext,
                                                frac_ext, spec_ext, sid_ext);
}
void launch_ghost_count(int n, const double* frac, const int* sid, const StructParams* sp,
                        int* count, hipStream_t s) {
  if (n > 0) k_ghost_count<<<nblk(n, 128), 128, 0, s>>>(n, frac, sid, sp, count);
}
void launch_ghost_fill(int n, const double* frac, const double* pos, const int* spec, int* sid,
                       const StructParams* sp, const int* gptr, int* owner, int* shift,
                       double* pos_ext, double* frac_ext, int* spec_ext, hipStream_t s) {
  if (n > 0)
    k_ghost_fill<<<nblk(n, 128), 128, 0, s>>>(n, frac, pos, spec, sid, sp, gptr, owner, shift,
                                              pos_ext, frac_ext, spec_ext);
}
void launch_bin_keys(int n, const double* frac, const int* sid, const StructParams* sp, int* key,
                     hipStream_t s) {
  if (n > 0) k_bin_keys<<<nblk(n, 256), 256, 0, s>>>(n, frac, sid, sp, key);
}
void launch_edge_count(int n, const double* pos_ext, const double* frac_ext, const int* sid,
                       const StructParams* sp, const int* cell_start, const int* cell_items,
                       double rc2, int* count, int* err, hipStream_t s) {
  if (n > 0)
    k_edges<false><<<nblk(n, 4), 256, 0, s>>>(n, pos_ext, frac_ext, sid, sp, cell_start,
                                                 cell_items, rc2, count, err, nullptr, nullptr,
                                                 nullptr);
}
void launch_edge_fill(int n, const double* pos_ext, const double* frac_ext, const int* sid,
                      const StructParams* sp, const int* cell_start, const int* cell_items,
                      double rc2, const int* row_ptr, int* src, int* recv, hipStream_t s) {
  if (n > 0)
    k_edges<true><<<nblk(n, 4), 256, 0, s>>>(n, pos_ext, frac_ext, sid, sp, cell_start,
                                                cell_items, rc2, nullptr, nullptr, row_ptr, src,
                                                recv);
}

}  // namespace sn

namespace sn {

// ------------------------------------------------------------------ reverse edges and pairs
// The reverse of e = (i <- s) is the edge of receiver o = owner(s) whose sender is an
// image of i shifted by -shift(s) (the local atom i itself when s is local).  Found by a
// scan of o's receiver segment; -1 when no such edge exists (possible only when the two
// directions round to different sides of r_c).
__global__ __launch_bounds__(256) void k_reverse(int64_t E, int n_local, const int* __restrict__ recv,
                                                 const int* __restrict__ src,
                                                 const int* __restrict__ row_ptr,
                                                 const int* __restrict__ owner,
                                                 const int* __restrict__ shift,
                                                 int* __restrict__ rev) {
  // 16 lanes per edge search o's segment together; the match is unique, the group keeps
  // the smallest index found
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int sub = threadIdx.x & 15;
  int found = INT_MAX;
  if (e < E) {
    const int i = recv[e], s = src[e];
    int o = s, sx = 0, sy = 0, sz = 0;
    if (s >= n_local) {
      const int g = s - n_local;
      o = owner[g];
      sx = shift[3 * g];
      sy = shift[3 * g + 1];
      sz = shift[3 * g + 2];
    }
    for (int q = row_ptr[o] + sub; q < row_ptr[o + 1]; q += 16) {
      const int t = src[q];
      bool match;
      if (t < n_local) {
        match = t == i && sx == 0 && sy == 0 && sz == 0;
      } else {
        const int g = t - n_local;
        match = owner[g] == i && shift[3 * g] == -sx && shift[3 * g + 1] == -sy &&
                shift[3 * g + 2] == -sz;
      }
      if (match) found = min(found, q);
    }
  }
  for (int off = 1; off < 16; off <<= 1) found = min(found, __shfl_xor(found, off));
  if (e < E && sub == 0) rev[e] = found == INT_MAX ? -1 : found;
}

__global__ void k_canon_flags(int64_t E, const int* __restrict__ rev, int* __restrict__ flag) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int r = rev[e];
  flag[e] = (r < 0 || e < r) ? 1 : 0;
}

__global__ void k_pairs(int64_t E, const int* __restrict__ rev, const int* __restrict__ flag,
                        const int* __restrict__ fscan, int* __restrict__ pidx,
                        int* __restrict__ pe1, int* __restrict__ pe2) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  // pidx[e] = 2 p + side: p is the undirected pair (row of the shared radial weights), side
  // 0 for the pair's first edge and 1 for its reverse (row 2p + side of the pair-major dE/dw)
  const int r = rev[e];
  if (flag[e]) {
    const int p = fscan[e];
    pidx[e] = 2 * p;
    pe1[p] = (int)e;
    pe2[p] = r;  // -1 when unpaired
  } else {
    pidx[e] = 2 * fscan[r] + 1;
  }
}

void launch_pairs(int64_t E, int n_local, const int* recv, const int* src, const int* row_ptr,
                  const int* owner, const int* shift, int* rev, int* flag, int* fscan, int* tmp,
                  int* pidx, int* pe1, int* pe2, hipStream_t s) {
  if (E <= 0) {
    k_scan_total<<<1, 1, 0, s>>>(flag, fscan, 0);
    return;
  }
  const unsigned g = (unsigned)((E + 255) / 256);
  k_reverse<<<(unsigned)((16 * E + 255) / 256), 256, 0, s>>>(E, n_local, recv, src, row_ptr,
                                                             owner, shift, rev);
  k_canon_flags<<<g, 256, 0, s>>>(E, rev, flag);
  scan_exclusive(flag, fscan, E, tmp, s);
  k_pairs<<<g, 256, 0, s>>>(E, rev, flag, fscan, pidx, pe1, pe2);
}

// ------------------------------------------------------------------ active-pair compaction
// A list built out to r_c + skin holds pairs whose atoms are now (or were at the build)
// farther apart than r_c.  The envelope vanishes there, so such an edge's radial weights,
// messages, sender gradients and edge gradient are exact zeros: the pairs inside r_c,
// compacted in order, give the same messages, energies and forces up to the grouping of
// floating-point sums.  A pair stays when either of its edges has r / r_c below 1 + 1e-12
// (the slack covers a last-bit difference from the edge-basis kernel's own distance).

__device__ inline bool edge_inside(const double* __restrict__ pos_ext, int i, int s, double r_cut) {
  const double d0 = pos_ext[3 * s] - pos_ext[3 * i];
  const double d1 = pos_ext[3 * s + 1] - pos_ext[3 * i + 1];
  const double d2 = pos_ext[3 * s + 2] - pos_ext[3 * i + 2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2) / r_cut < 1.0 + 1e-12;
}

__global__ void k_pair_active(int64_t np, const int* __restrict__ pe1, const int* __restrict__ pe2,
                              const int* __restrict__ recv, const int* __restrict__ src,
                              const double* __restrict__ pos_ext, double r_cut,
                              int* __restrict__ active) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int e1 = pe1[p], e2 = pe2[p];
  bool in = edge_inside(pos_ext, recv[e1], src[e1], r_cut);
  if (!in && e2 >= 0) in = edge_inside(pos_ext, recv[e2], src[e2], r_cut);
  active[p] = in ? 1 : 0;
}

// keep[e] for every edge, and keep_s[k] for every entry of the sender list
__global__ void k_edge_keep(int64_t E, const int* __restrict__ pidx, const int* __restrict__ active,
                            const int* __restrict__ send_idx, int* __restrict__ keep,
                            int* __restrict__ keep_s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  keep[e] = active[pidx[e] >> 1];
  keep_s[e] = active[pidx[send_idx[e]] >> 1];
}

__global__ void k_compact_edges(int64_t E, const int* __restrict__ keep, const int* __restrict__ escan,
                                const int* __restrict__ pscan, const int* __restrict__ src,
                                const int* __restrict__ recv, const int* __restrict__ pidx,
                                const int* __restrict__ send_idx, const int* __restrict__ keep_s,
                                const int* __restrict__ sscan, int* __restrict__ src_o,
                                int* __restrict__ recv_o, int* __restrict__ pidx_o,
                                int* __restrict__ send_idx_o) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  if (keep[e]) {
    const int ne = escan[e], q = pidx[e];
    src_o[ne] = src[e];
    recv_o[ne] = recv[e];
    pidx_o[ne] = 2 * pscan[q >> 1] + (q & 1);
  }
  if (keep_s[e]) send_idx_o[sscan[e]] = escan[send_idx[e]];
}

__global__ void k_compact_pairs(int64_t np, const int* __restrict__ active, const int* __restrict__ pscan,
                                const int* __restrict__ escan, const int* __restrict__ pe1,
                                const int* __restrict__ pe2, int* __restrict__ pe1_o,
                                int* __restrict__ pe2_o) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np || !active[p]) return;
  const int q = pscan[p];
  pe1_o[q] = escan[pe1[p]];
  pe2_o[q] = pe2[p] >= 0 ? escan[pe2[p]] : -1;
}

// out[k] = scan[in[k]] for k <= n (segment offsets of the compacted arrays)
__global__ void k_remap_offsets(int n, const int* __restrict__ in, const int* __restrict__ scan,
                                int* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= n) out[k] = scan[in[k]];
}

void launch_compact_active(const CompactIn& a, const CompactOut& o, CompactScratch& t,
                           hipStream_t s) {
  const unsigned gp = (unsigned)((a.np + 255) / 256), ge = (unsigned)((a.E + 255) / 256);
  if (a.np > 0)
    k_pair_active<<<gp, 256, 0, s>>>(a.np, a.pe1, a.pe2, a.recv, a.src, a.pos_ext, a.r_cut,
                                     t.active);
  scan_exclusive(t.active, t.pscan, a.np, t.tmp, s);
  if (a.E > 0) k_edge_keep<<<ge, 256, 0, s>>>(a.E, a.pidx, t.active, a.send_idx, t.keep, t.keep_s);
  scan_exclusive(t.keep, t.escan, a.E, t.tmp, s);
  scan_exclusive(t.keep_s, t.sscan, a.E, t.tmp, s);
  if (a.E > 0)
    k_compact_edges<<<ge, 256, 0, s>>>(a.E, t.keep, t.escan, t.pscan, a.src, a.recv, a.pidx,
                                       a.send_idx, t.keep_s, t.sscan, o.src, o.recv, o.pidx,
                                       o.send_idx);
  if (a.np > 0)
    k_compact_pairs<<<gp, 256, 0, s>>>(a.np, t.active, t.pscan, t.escan, a.pe1, a.pe2, o.pe1,
                                       o.pe2);
  k_remap_offsets<<<(unsigned)((a.n_local + 1 + 255) / 256), 256, 0, s>>>(a.n_local, a.row_ptr,
                                                                           t.escan, o.row_ptr);
  k_remap_offsets<<<(unsigned)((a.n_ext + 1 + 255) / 256), 256, 0, s>>>(a.n_ext, a.send_ptr,
                                                                         t.sscan, o.send_ptr);
  k_remap_offsets<<<(unsigned)((a.n_struct + 1 + 255) / 256), 256, 0, s>>>(a.n_struct, a.edge_off,
                                                                            t.escan, o.edge_off);
}

}  // namespace sn
