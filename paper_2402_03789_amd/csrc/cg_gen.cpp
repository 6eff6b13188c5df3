// Build-time generator of the real Clebsch-Gordan coupling tensors used by
// the tensor-product kernels (the convolution block of the NequIP
// interaction block, paper section 2.2; spherical harmonics up to l = 2 for the
// model of section 5.1 and up to l = 3 for the benchmark models of section 4).
//
// Method: the coupling C[m1][m2][m3] of degrees (l1, l2) into l3 is the
// one-dimensional null space of the equivariance equations
//     sum_{a,b} C[a][b][c] D1[a][a'] D2[b][b'] - sum_{c'} D3[c][c'] C[a'][b'][c'] = 0
// for two random rotations, where D_l are the real Wigner matrices of the
// harmonic basis Y^l used on edges (fitted from Y^l evaluated at rotated
// sample points).  The solution is normalised so that
// sum_{a,b} C[a][b][c] C[a][b][c'] = delta(c, c'), and its sign is fixed so
// that the first nonzero entry in row-major (m1, m2, m3) order is positive.
//
// Output: a header with, for each (l1, l2, l3) with l <= 3, a struct whose
// static `each(f)` calls f(m1, m2, m3, value) for every nonzero entry, and a
// dense table used by the library's table-export entry point.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include <string>

static void sh(int l, const double v[3], double* out) {
  const double x = v[0], y = v[1], z = v[2];
  if (l == 0) {
    out[0] = 1.0;
  } else if (l == 1) {
    const double s3 = std::sqrt(3.0);
    out[0] = s3 * y; out[1] = s3 * z; out[2] = s3 * x;
  } else if (l == 2) {
    const double s15 = std::sqrt(15.0), s5 = std::sqrt(5.0);
    out[0] = s15 * x * y;
    out[1] = s15 * y * z;
    out[2] = 0.5 * s5 * (3.0 * z * z - 1.0);
    out[3] = s15 * x * z;
    out[4] = 0.5 * s15 * (x * x - y * y);
  } else {  // l = 3, on the unit sphere
    const double a = std::sqrt(70.0) / 4, b = std::sqrt(105.0), c = std::sqrt(42.0) / 4,
                 d = std::sqrt(7.0) / 2;
    out[0] = a * y * (3.0 * x * x - y * y);
    out[1] = b * x * y * z;
    out[2] = c * y * (5.0 * z * z - 1.0);
    out[3] = d * z * (5.0 * z * z - 3.0);
    out[4] = c * x * (5.0 * z * z - 1.0);
    out[5] = 0.5 * b * z * (x * x - y * y);
    out[6] = a * x * (x * x - 3.0 * y * y);
  }
}

constexpr int kL = 3;  // highest degree generated

// Solve A X = B (n x n, n x m) by Gaussian elimination with partial pivoting.
static void solve(int n, int m, std::vector<double> A, std::vector<double>& B) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r) if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
    for (int k = 0; k < m; ++k) std::swap(B[c * m + k], B[p * m + k]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c] / A[c * n + c];
      for (int k = 0; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < m; ++k) B[r * m + k] -= f * B[c * m + k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < m; ++k) B[r * m + k] /= A[r * n + r];
}

// Real Wigner matrix D (d x d) with Y(R v) = D Y(v), least squares over samples.
static std::vector<double> wigner(int l, const double R[9], std::mt19937_64& g) {
  const int d = 2 * l + 1, S = 24;
  std::normal_distribution<double> nd;
  std::vector<double> Y(S * d), Yr(S * d);
  for (int s = 0; s < S; ++s) {
    double v[3] = {nd(g), nd(g), nd(g)};
    double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (double& c : v) c /= nrm;
    double w[3];
    for (int i = 0; i < 3; ++i) w[i] = R[i * 3] * v[0] + R[i * 3 + 1] * v[1] + R[i * 3 + 2] * v[2];
    sh(l, v, &Y[s * d]);
    sh(l, w, &Yr[s * d]);
  }
  // normal equations: (Y^T Y) D^T = Y^T Yr
  std::vector<double> A(d * d, 0.0), B(d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      for (int s = 0; s < S; ++s) {
        A[i * d + j] += Y[s * d + i] * Y[s * d + j];
        B[i * d + j] += Y[s * d + i] * Yr[s * d + j];
      }
  solve(d, d, A, B);  // B = D^T
  std::vector<double> D(d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) D[i * d + j] = B[j * d + i];
  return D;
}

static void random_rotation(std::mt19937_64& g, double R[9]) {
  std::normal_distribution<double> nd;
  double q[4] = {nd(g), nd(g), nd(g), nd(g)};
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (double& c : q) c /= n;
  double w = q[0], x = q[1], y = q[2], z = q[3];
  double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                 2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                 2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
  for (int i = 0; i < 9; ++i) R[i] = M[i];
}

// One-dimensional null space of K (rows x n) by elimination with full pivoting.
static std::vector<double> null_vector(int rows, int n, std::vector<double> K) {
  std::vector<int> colperm(n);
  for (int i = 0; i < n; ++i) colperm[i] = i;
  int rank = 0;
  for (int c = 0; c < n && rank < rows; ++c) {
    int br = -1, bc = -1;
    double best = 0;
    for (int r = rank; r < rows; ++r)
      for (int k = c; k < n; ++k)
        if (std::fabs(K[r * n + k]) > best) { best = std::fabs(K[r * n + k]); br = r; bc = k; }
    if (best < 1e-9) break;
    for (int k = 0; k < n; ++k) std::swap(K[rank * n + k], K[br * n + k]);
    for (int r = 0; r < rows; ++r) std::swap(K[r * n + c], K[r * n + bc]);
    std::swap(colperm[c], colperm[bc]);
    double piv = K[rank * n + c];
    for (int k = 0; k < n; ++k) K[rank * n + k] /= piv;
    for (int r = 0; r < rows; ++r) {
      if (r == rank) continue;
      double f = K[r * n + c];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) K[r * n + k] -= f * K[rank * n + k];
    }
    ++rank;
  }
  if (rank != n - 1) {
    std::fprintf(stderr, "cg_gen: null space has dimension %d\n", n - rank);
    std::exit(1);
  }
  // free column is n-1 (after permutation): x_free = 1, x_pivot_r = -K[r][n-1]
  std::vector<double> xp(n);
  for (int r = 0; r < n - 1; ++r) xp[r] = -K[r * n + (n - 1)];
  xp[n - 1] = 1.0;
  std::vector<double> x(n);
  for (int i = 0; i < n; ++i) x[colperm[i]] = xp[i];
  return x;
}

int main(int argc, char** argv) {
  const char* out_path = argc > 1 ? argv[1] : "cg_tables.h";
  std::mt19937_64 g(20240206ULL);
  double R[2][9];
  random_rotation(g, R[0]);
  random_rotation(g, R[1]);
  std::vector<double> D[2][kL + 1];
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l <= kL; ++l) D[k][l] = wigner(l, R[k], g);

  int n_triples = 0;
  for (int l1 = 0; l1 <= kL; ++l1)
    for (int l2 = 0; l2 <= kL; ++l2)
      for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, kL); ++l3) ++n_triples;
  const int dmax = (2 * kL + 1) * (2 * kL + 1) * (2 * kL + 1);
  std::string hdr;
  char line[256];
  hdr += "// Generated by cg_gen.cpp: real Clebsch-Gordan coupling tensors, l <= 3.\n";
  hdr += "// Do not edit.\n#pragma once\n\nnamespace sn {\n\n";
  std::snprintf(line, sizeof line, "constexpr int kCGMaxL = %d;\nconstexpr int kCGTriples = %d;\n\n",
                kL, n_triples);
  hdr += line;
  hdr += "template <int L1, int L2, int L3> struct CG;\n\n";
  std::snprintf(line, sizeof line, "static const double kCGDense[%d][%d] = {\n", n_triples, dmax);
  std::string dense = line;
  int path_id = 0;
  int total_nnz = 0;
  for (int l1 = 0; l1 <= kL; ++l1)
    for (int l2 = 0; l2 <= kL; ++l2)
      for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, kL); ++l3) {
        const int d1 = 2 * l1 + 1, d2 = 2 * l2 + 1, d3 = 2 * l3 + 1, n = d1 * d2 * d3;
        std::vector<double> K;
        for (int k = 0; k < 2; ++k) {
          const auto &A1 = D[k][l1], &A2 = D[k][l2], &A3 = D[k][l3];
          for (int ap = 0; ap < d1; ++ap)
            for (int bp = 0; bp < d2; ++bp)
              for (int c = 0; c < d3; ++c) {
                std::vector<double> row(n, 0.0);
                for (int a = 0; a < d1; ++a)
                  for (int b = 0; b < d2; ++b) row[(a * d2 + b) * d3 + c] += A1[a * d1 + ap] * A2[b * d2 + bp];
                for (int cp = 0; cp < d3; ++cp) row[(ap * d2 + bp) * d3 + cp] -= A3[c * d3 + cp];
                K.insert(K.end(), row.begin(), row.end());
              }
        }
        std::vector<double> C = null_vector((int)(K.size() / n), n, K);
        double nrm = 0;
        for (int a = 0; a < d1; ++a)
          for (int b = 0; b < d2; ++b) nrm += C[(a * d2 + b) * d3] * C[(a * d2 + b) * d3];
        nrm = std::sqrt(nrm);
        for (double& c : C) c /= nrm;
        int first = -1;
        for (int i = 0; i < n; ++i) {
          if (std::fabs(C[i]) < 1e-10) C[i] = 0.0;
          if (first < 0 && C[i] != 0.0) first = i;
        }
        if (C[first] < 0) for (double& c : C) c = -c;
        char buf[256];
        std::snprintf(buf, sizeof buf, "template <> struct CG<%d, %d, %d> {\n", l1, l2, l3);
        hdr += buf;
        hdr += "  template <class F> __host__ __device__ static inline void each(F&& f) {\n";
        int nnz = 0;
        for (int a = 0; a < d1; ++a)
          for (int b = 0; b < d2; ++b)
            for (int c = 0; c < d3; ++c) {
              double v = C[(a * d2 + b) * d3 + c];
              if (v == 0.0) continue;
              std::snprintf(buf, sizeof buf, "    f(%d, %d, %d, %.17g);\n", a, b, c, v);
              hdr += buf;
              ++nnz;
            }
        total_nnz += nnz;
        std::snprintf(buf, sizeof buf, "  }\n  static constexpr int nnz = %d;\n};\n\n", nnz);
        hdr += buf;
        dense += "  {";
        for (int i = 0; i < dmax; ++i) {
          std::snprintf(buf, sizeof buf, "%.17g%s", i < n ? C[i] : 0.0, i < dmax - 1 ? ", " : "");
          dense += buf;
        }
        dense += "},\n";
        ++path_id;
      }
  dense += "};\n";
  hdr += dense;
  hdr += "\n}  // namespace sn\n";
  FILE* f = std::fopen(out_path, "w");
  if (!f) { std::perror(out_path); return 1; }
  std::fputs(hdr.c_str(), f);
  std::fclose(f);
  std::fprintf(stderr, "cg_gen: %d paths, %d nonzeros -> %s\n", path_id, total_nnz, out_path);
  return 0;
}
