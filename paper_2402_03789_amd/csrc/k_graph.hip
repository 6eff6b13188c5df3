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

// insertion sort of each segment (segments are short: bin or sender lists)
__global__ void k_sort_segments(int nseg, const int* __restrict__ start, int* __restrict__ items) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int a = start[s], b = start[s + 1];
  for (int i = a + 1; i < b; ++i) {
    int v = items[i];
    int j = i - 1;
    while (j >= a && items[j] > v) {
      items[j + 1] = items[j];
      --j;
    }
    items[j + 1] = v;
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
  const BinGrid& g0 = P.g;
  for (int d = P.first_region; d < P.first_region + nreg; ++d) {
    const BinGrid& g = sp[d].g;
    for (int sx = -g0.nimg[0]; sx <= g0.nimg[0]; ++sx)
      for (int sy = -g0.nimg[1]; sy <= g0.nimg[1]; ++sy)
        for (int sz = -g0.nimg[2]; sz <= g0.nimg[2]; ++sz) {
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

template <bool FILL>
__global__ void k_edges(int n, const double* __restrict__ pos_ext, const double* __restrict__ frac_ext,
                        const int* __restrict__ sid, const StructParams* __restrict__ sp,
                        const int* __restrict__ cell_start, const int* __restrict__ cell_items,
                        double rc2, int* __restrict__ count, int* __restrict__ err,
                        const int* __restrict__ row_ptr, int* __restrict__ src,
                        int* __restrict__ recv) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const StructParams& P = sp[sid[k]];
  const BinGrid& g = P.g;
  double p[3] = {pos_ext[3 * k], pos_ext[3 * k + 1], pos_ext[3 * k + 2]};
  double f[3] = {frac_ext[3 * k], frac_ext[3 * k + 1], frac_ext[3 * k + 2]};
  int b[3];
  for (int a = 0; a < 3; ++a) b[a] = bin_axis(f[a], g, a);
  int c = 0;
  int w = FILL ? row_ptr[k] : 0;
  for (int bx = max(b[0] - 1, 0); bx <= min(b[0] + 1, g.nb[0] - 1); ++bx)
    for (int by = max(b[1] - 1, 0); by <= min(b[1] + 1, g.nb[1] - 1); ++by)
      for (int bz = max(b[2] - 1, 0); bz <= min(b[2] + 1, g.nb[2] - 1); ++bz) {
        int cell = P.bin_base + (bx * g.nb[1] + by) * g.nb[2] + bz;
        for (int q = cell_start[cell]; q < cell_start[cell + 1]; ++q) {
          int s = cell_items[q];
          if (s == k) continue;
          double dx = pos_ext[3 * s] - p[0], dy = pos_ext[3 * s + 1] - p[1],
                 dz = pos_ext[3 * s + 2] - p[2];
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < rc2) {
            if (!FILL && r2 < 1e-16) atomicOr(err, 2);
            if (FILL) {
              src[w] = s;
              recv[w] = k;
              ++w;
            } else {
              ++c;
            }
          }
        }
      }
  if (!FILL) count[k] = c;
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
  if (nseg > 0) k_sort_segments<<<nblk(nseg, 128), 128, 0, s>>>(nseg, start, items);
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
    k_edges<false><<<nblk(n, 128), 128, 0, s>>>(n, pos_ext, frac_ext, sid, sp, cell_start,
                                                 cell_items, rc2, count, err, nullptr, nullptr,
                                                 nullptr);
}
void launch_edge_fill(int n, const double* pos_ext, const double* frac_ext, const int* sid,
                      const StructParams* sp, const int* cell_start, const int* cell_items,
                      double rc2, const int* row_ptr, int* src, int* recv, hipStream_t s) {
  if (n > 0)
    k_edges<true><<<nblk(n, 128), 128, 0, s>>>(n, pos_ext, frac_ext, sid, sp, cell_start,
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
__global__ void k_reverse(int64_t E, int n_local, const int* __restrict__ recv,
                          const int* __restrict__ src, const int* __restrict__ row_ptr,
                          const int* __restrict__ owner, const int* __restrict__ shift,
                          int* __restrict__ rev) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int i = recv[e], s = src[e];
  int o = s, sx = 0, sy = 0, sz = 0;
  if (s >= n_local) {
    const int g = s - n_local;
    o = owner[g];
    sx = shift[3 * g];
    sy = shift[3 * g + 1];
    sz = shift[3 * g + 2];
  }
  int found = -1;
  for (int q = row_ptr[o]; q < row_ptr[o + 1]; ++q) {
    const int t = src[q];
    if (t < n_local) {
      if (t == i && sx == 0 && sy == 0 && sz == 0) { found = q; break; }
    } else {
      const int g = t - n_local;
      if (owner[g] == i && shift[3 * g] == -sx && shift[3 * g + 1] == -sy &&
          shift[3 * g + 2] == -sz) { found = q; break; }
    }
  }
  rev[e] = found;
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
  k_reverse<<<g, 256, 0, s>>>(E, n_local, recv, src, row_ptr, owner, shift, rev);
  k_canon_flags<<<g, 256, 0, s>>>(E, rev, flag);
  scan_exclusive(flag, fscan, E, tmp, s);
  k_pairs<<<g, 256, 0, s>>>(E, rev, flag, fscan, pidx, pe1, pe2);
}

}  // namespace sn
