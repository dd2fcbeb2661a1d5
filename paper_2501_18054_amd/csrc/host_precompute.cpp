// Host precompute of libpngf (FP64, OpenMP, AVX2): the once-only folding of
// the static environment into the design-region Green function.
//
// Results, Precomputation: G = B^T A^-1 B over the optimization region is the
// negated Schur complement of the augmented system [[A, B], [B^T, 0]]; the
// paper obtains it with a partial factorization (APF) that eliminates every
// unknown outside the region first.  The same idea is applied here to the 2D
// TM FDFD operator, in two stages, both ordered by nested dissection:
//
//   * A = S L is the complex-symmetric, PML-scaled 5-point operator
//     (S = diag(s_x s_y), which is 1 away from the PML).  The source
//     f = S i k0 J and the output functional w are appended as two extra
//     columns (and rows) of A, so that every elimination also carries them.
//   * Stage 1 (exterior, multifrontal): the exterior nodes O are eliminated
//     by a geometric nested dissection of the grid (boxes split by a grid
//     line; the line is the box's separator).  Each box's front holds its
//     separator, its boundary nodes and the two extra columns; eliminating the
//     separator leaves a Schur update on the boundary that is added into the
//     parent's front.  What remains at the root is, on the design pixels D,
//        S_D  = A_DD - A_DO A_OO^-1 A_OD           (dense on the perimeter)
//        r_D  = f_D  - A_DO A_OO^-1 f_O,   v = w_D - A_DO A_OO^-1 w_O,
//        c    = w_O^T A_OO^-1 f_O.
//   * Stage 2 (design region): G = -(S_D)^-1 by block sweeps (block
//     Gauss-Jordan steps on a symmetric matrix: sweeping every index of a
//     matrix leaves minus its inverse).  The pixels are ordered by a nested
//     dissection of the interior with the perimeter last; a box's separator
//     couples only to the box and its boundary, so its sweep touches only
//     those rows, and most of the work is the last (perimeter) sweep, a
//     rank-|perimeter| update of the whole matrix.
//   * Then b = E_b[D] = S_D^-1 r_D = -G r_D, G_OD = v^T G (reciprocity),
//     x_b = c + v^T b.
//
// The objective normalizer of the mean-transmission objective is
// |w^T E_hom|^2 with E_hom the field of the same source in vacuum (eps = 1
// on the whole grid, no design): stage 1 with no kept node gives it.
//
// Every dense step is a block elimination whose pivot block is inverted by
// Gauss-Jordan with partial pivoting; the rank-b updates run on a register-
// blocked complex GEMM kernel (AVX2 + FMA).
//
// The discrete problem (the same one the CPU oracle states independently):
//   d(u) = max(0, npml-u, u-(N-1-npml))/npml, sigma = sigma_max d^3,
//   sigma_max = -(3+1) ln(1e-8) / (2 npml h), s(u) = 1 - i sigma(u)/k0,
//   L E = [D_x (1/s_x) D_x / s_x + D_y (1/s_y) D_y / s_y + k0^2 eps] E = i k0 J,
//   Ez = 0 beyond the grid.
#include <immintrin.h>
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "pngf_internal.h"

namespace pngf {

namespace {

constexpr double kPmlLnR = -18.420680743952367;  // ln(1e-8)
constexpr double kPmlOrder = 3.0;

struct Stretch {
  int n, npml;
  double h, k0;
  cd at(double u) const {
    if (npml <= 0) return cd(1.0, 0.0);
    double d = std::max(0.0, std::max(npml - u, u - (n - 1 - npml))) / npml;
    double smax = -(kPmlOrder + 1.0) * kPmlLnR / (2.0 * npml * h);
    double sigma = smax * d * d * d;
    return cd(1.0, -sigma / k0);
  }
};

// Complex-symmetric operator A = S L on the grid: diagonal, +x link, +y link.
struct Operator {
  int nx, ny;
  std::vector<cd> diag, xl, yl;  // xl[n]: (n, n+1); yl[n]: (n, n+nx)
  std::vector<cd> scale;         // S = s_x(i) s_y(j)
};

Operator build_operator(const Grid& g, const std::vector<double>& eps, double k0) {
  Operator op;
  op.nx = g.nx;
  op.ny = g.ny;
  const int64_t N = int64_t(g.nx) * g.ny;
  op.diag.assign(N, 0.0);
  op.xl.assign(N, 0.0);
  op.yl.assign(N, 0.0);
  op.scale.assign(N, 0.0);
  Stretch sx{g.nx, g.npml, g.h, k0}, sy{g.ny, g.npml, g.h, k0};
  const double ih2 = 1.0 / (g.h * g.h);
  for (int j = 0; j < g.ny; ++j) {
    cd syn = sy.at(j), syp = sy.at(j + 0.5), sym = sy.at(j - 0.5);
    for (int i = 0; i < g.nx; ++i) {
      cd sxn = sx.at(i), sxp = sx.at(i + 0.5), sxm = sx.at(i - 0.5);
      int64_t n = int64_t(j) * g.nx + i;
      op.scale[n] = sxn * syn;
      op.diag[n] = k0 * k0 * eps[n] * sxn * syn - syn * (1.0 / sxp + 1.0 / sxm) * ih2 -
                   sxn * (1.0 / syp + 1.0 / sym) * ih2;
      if (i + 1 < g.nx) op.xl[n] = syn / sxp * ih2;
      if (j + 1 < g.ny) op.yl[n] = sxn / syp * ih2;
    }
  }
  return op;
}

// Coupling A(n, m) of two 4-neighbours n, m (either order).
inline cd link(const Operator& op, int64_t n, int64_t m) {
  const int64_t lo = std::min(n, m), d = std::max(n, m) - lo;
  return d == 1 ? op.xl[lo] : op.yl[lo];
}

// ------------------------------------------------------------ dense kernels
//
// All matrices are row-major std::complex<double> (interleaved re, im).
// gemm_nt: C (m x n) = or -= A (m x k) Bt^T with Bt (n x k): both operands
// are read along k.  Bt is packed per panel of kNc columns into groups of
// four columns: for every k the four values (re, im) and the four rotated
// values (-im, re), so that a*b = re(a) b + im(a) rot(b) is two FMAs with
// broadcast re(a), im(a).  The micro-tile is 4 rows x 4 complex columns
// (8 accumulators of 2 complex each).

constexpr int kNc = 128;  // columns per packed panel
constexpr int kMb = 32;   // rows per task

void pack_bt(const cd* Bt, int64_t ldb, int j0, int nc, int k, double* out) {
  const int ng = (nc + 3) / 4;
  for (int g = 0; g < ng; ++g) {
    double* o = out + int64_t(g) * k * 16;
    for (int t = 0; t < 4; ++t) {
      const int jj = 4 * g + t;
      if (jj < nc) {
        const double* src = reinterpret_cast<const double*>(Bt + int64_t(j0 + jj) * ldb);
        for (int kk = 0; kk < k; ++kk) {
          const double re = src[2 * kk], im = src[2 * kk + 1];
          double* ok = o + int64_t(kk) * 16;
          ok[2 * t] = re;
          ok[2 * t + 1] = im;
          ok[8 + 2 * t] = -im;
          ok[8 + 2 * t + 1] = re;
        }
      } else {
        for (int kk = 0; kk < k; ++kk) {
          double* ok = o + int64_t(kk) * 16;
          ok[2 * t] = ok[2 * t + 1] = ok[8 + 2 * t] = ok[8 + 2 * t + 1] = 0.0;
        }
      }
    }
  }
}

template <int MR>
inline void micro_nt(int k, const double* a, int64_t lda2, const double* bp, double* c,
                     int64_t ldc2, int ncol, bool assign) {
  __m256d acc[MR][2];
#pragma unroll
  for (int r = 0; r < MR; ++r) acc[r][0] = acc[r][1] = _mm256_setzero_pd();
  for (int kk = 0; kk < k; ++kk) {
    const double* b = bp + int64_t(kk) * 16;
    const __m256d b0 = _mm256_loadu_pd(b), b1 = _mm256_loadu_pd(b + 4);
    const __m256d s0 = _mm256_loadu_pd(b + 8), s1 = _mm256_loadu_pd(b + 12);
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const __m256d ar = _mm256_broadcast_sd(a + r * lda2 + 2 * kk);
      const __m256d ai = _mm256_broadcast_sd(a + r * lda2 + 2 * kk + 1);
      acc[r][0] = _mm256_fmadd_pd(ar, b0, acc[r][0]);
      acc[r][1] = _mm256_fmadd_pd(ar, b1, acc[r][1]);
      acc[r][0] = _mm256_fmadd_pd(ai, s0, acc[r][0]);
      acc[r][1] = _mm256_fmadd_pd(ai, s1, acc[r][1]);
    }
  }
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    double* cr = c + r * ldc2;
    if (ncol == 4) {
      if (assign) {
        _mm256_storeu_pd(cr, acc[r][0]);
        _mm256_storeu_pd(cr + 4, acc[r][1]);
      } else {
        _mm256_storeu_pd(cr, _mm256_sub_pd(_mm256_loadu_pd(cr), acc[r][0]));
        _mm256_storeu_pd(cr + 4, _mm256_sub_pd(_mm256_loadu_pd(cr + 4), acc[r][1]));
      }
    } else {
      alignas(32) double t[8];
      _mm256_store_pd(t, acc[r][0]);
      _mm256_store_pd(t + 4, acc[r][1]);
      for (int q = 0; q < 2 * ncol; ++q) cr[q] = assign ? t[q] : cr[q] - t[q];
    }
  }
}

// C (m x n) op= A Bt^T.  assign: C = A Bt^T, else C -= A Bt^T.  lower: only
// the entries with j <= i are needed; 4x4 tiles that lie wholly above the
// diagonal are skipped (tiles crossing it are written whole).
void gemm_nt(int m, int n, int k, const cd* A, int64_t lda, const cd* Bt, int64_t ldb, cd* C,
             int64_t ldc, bool assign, bool lower, int nt) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {
    if (assign)
      for (int i = 0; i < m; ++i) std::fill(C + int64_t(i) * ldc, C + int64_t(i) * ldc + n, cd(0.0));
    return;
  }
  std::vector<double> bp(size_t((kNc + 3) / 4) * k * 16);
  const double* a2 = reinterpret_cast<const double*>(A);
  double* c2 = reinterpret_cast<double*>(C);
  for (int j0 = 0; j0 < n; j0 += kNc) {
    const int nc = std::min(kNc, n - j0);
    pack_bt(Bt, ldb, j0, nc, k, bp.data());
    const int i0 = lower ? std::min(j0, m) : 0;
    const int nblk = (m - i0 + kMb - 1) / kMb;
    const double work = double(m - i0) * nc * k;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt) if (nt > 1 && nblk > 1 && work > 4e5)
    for (int blk = 0; blk < nblk; ++blk) {
      const int ib = i0 + blk * kMb, ie = std::min(m, ib + kMb);
      for (int g = 0; 4 * g < nc; ++g) {
        const int jg = j0 + 4 * g;
        if (lower && jg > ie - 1) break;
        const int ncol = std::min(4, nc - 4 * g);
        const double* bg = bp.data() + int64_t(g) * k * 16;
        for (int i = ib; i < ie; i += 4) {
          const int mr = std::min(4, ie - i);
          if (lower && jg > i + mr - 1) continue;
          const double* ai = a2 + 2 * int64_t(i) * lda;
          double* ci = c2 + 2 * (int64_t(i) * ldc + jg);
          switch (mr) {
            case 4: micro_nt<4>(k, ai, 2 * lda, bg, ci, 2 * ldc, ncol, assign); break;
            case 3: micro_nt<3>(k, ai, 2 * lda, bg, ci, 2 * ldc, ncol, assign); break;
            case 2: micro_nt<2>(k, ai, 2 * lda, bg, ci, 2 * ldc, ncol, assign); break;
            default: micro_nt<1>(k, ai, 2 * lda, bg, ci, 2 * ldc, ncol, assign); break;
          }
        }
      }
    }
  }
}

// In-place inverse of a dense complex n x n matrix by Gauss-Jordan elimination
// with partial pivoting; nt threads for the row updates.
int gj_inverse(cd* a, int n, int64_t ld, int nt) {
  std::vector<int> piv(n);
  std::vector<cd> rowk(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(a[int64_t(k) * ld + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::abs(a[int64_t(i) * ld + k]);
      if (v > best) { best = v; p = i; }
    }
    if (!(best > 0.0) || !std::isfinite(best)) return PNGF_ESINGULAR;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[int64_t(k) * ld + j], a[int64_t(p) * ld + j]);
    cd* ak = &a[int64_t(k) * ld];
    const cd inv = 1.0 / ak[k];
    ak[k] = 1.0;
    for (int j = 0; j < n; ++j) ak[j] *= inv;
    std::memcpy(rowk.data(), ak, sizeof(cd) * n);
    const double* rk = reinterpret_cast<const double*>(rowk.data());
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1 && n > 256)
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      cd* ai = &a[int64_t(i) * ld];
      const cd f = ai[k];
      if (f == cd(0.0, 0.0)) continue;
      ai[k] = 0.0;
      const double fr = f.real(), fi = f.imag();
      double* r = reinterpret_cast<double*>(ai);
      for (int j = 0; j < n; ++j) {
        const double xr = rk[2 * j], xi = rk[2 * j + 1];
        r[2 * j] -= fr * xr - fi * xi;
        r[2 * j + 1] -= fr * xi + fi * xr;
      }
    }
  }
  // Undo the row interchanges as column interchanges, last first.
  for (int k = n - 1; k >= 0; --k) {
    if (piv[k] == k) continue;
    const int p = piv[k];
    for (int i = 0; i < n; ++i) std::swap(a[int64_t(i) * ld + k], a[int64_t(i) * ld + p]);
  }
  return PNGF_OK;
}

// Block elimination of the last b indices of the complex-symmetric m x m
// matrix W (lower triangle stored, row-major, leading dimension ld), with
// nb = m - b, B the last b indices and Bi = W_BB^-1 (Gauss-Jordan, partial
// pivoting, then symmetrized):
//   W[0:nb, 0:nb] -= W[0:nb, B] Bi W[B, 0:nb]          (the Schur update)
// and, if sweep, the block sweep of B:
//   W[B, 0:nb] = (W[0:nb, B] Bi)^T,   W_BB = -Bi.
// Sweeping every index of a symmetric matrix, block by block in any order,
// leaves minus its inverse.
int eliminate_last(cd* W, int m, int64_t ld, int b, bool sweep, int nt) {
  if (b <= 0) return PNGF_OK;
  const int nb = m - b;
  std::vector<cd> Bi(size_t(b) * b);
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < b; ++c)
      Bi[size_t(r) * b + c] = W[int64_t(nb + std::max(r, c)) * ld + nb + std::min(r, c)];
  int st = gj_inverse(Bi.data(), b, b, nt);
  if (st != PNGF_OK) return st;
  for (int r = 0; r < b; ++r)
    for (int c = 0; c < r; ++c) {
      const cd s = 0.5 * (Bi[size_t(r) * b + c] + Bi[size_t(c) * b + r]);
      Bi[size_t(r) * b + c] = s;
      Bi[size_t(c) * b + r] = s;
    }
  if (nb > 0) {
    // Pn[i][k] = W[i][nb+k] = W[nb+k][i] (lower); Q = Pn Bi (Bi symmetric).
    std::vector<cd> Pn(size_t(nb) * b), Q(size_t(nb) * b);
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1 && int64_t(nb) * b > 65536)
    for (int i = 0; i < nb; ++i)
      for (int kk = 0; kk < b; ++kk) Pn[size_t(i) * b + kk] = W[int64_t(nb + kk) * ld + i];
    gemm_nt(nb, b, b, Pn.data(), b, Bi.data(), b, Q.data(), b, true, false, nt);
    gemm_nt(nb, nb, b, Q.data(), b, Pn.data(), b, W, ld, false, true, nt);
    if (sweep) {
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1 && int64_t(nb) * b > 65536)
      for (int kk = 0; kk < b; ++kk)
        for (int i = 0; i < nb; ++i) W[int64_t(nb + kk) * ld + i] = Q[size_t(i) * b + kk];
    }
  }
  if (sweep)
    for (int r = 0; r < b; ++r)
      for (int c = 0; c <= r; ++c) W[int64_t(nb + r) * ld + nb + c] = -Bi[size_t(r) * b + c];
  return PNGF_OK;
}

// ------------------------------------------------------- nested dissection
//
// Node classes on the grid: 0 = absent, 1 = eliminated through the tree,
// 2 = kept (never eliminated here).  A tree node is a box [x0,x1) x [y0,y1)
// of the grid; its members are the class-1 nodes in the box.  An inner node
// is split by the grid line through its middle (across its longer side): the
// class-1 nodes on that line are its separator, the two sides its children.
// A leaf (at most kLeaf members) has all its members as separator.  Nodes are
// stored children first (postorder).

constexpr int kLeaf = 64;

struct NdNode {
  int x0, y0, x1, y1;
  std::vector<int64_t> sep;  // flat grid ids, row-major
  int child[2] = {-1, -1};
};

int nd_build(std::vector<NdNode>& t, const Grid& g, const std::vector<uint8_t>& cls, int x0,
             int y0, int x1, int y1) {
  if (x1 <= x0 || y1 <= y0) return -1;
  int64_t cnt = 0;
  for (int j = y0; j < y1; ++j)
    for (int i = x0; i < x1; ++i) cnt += cls[int64_t(j) * g.nx + i] == 1;
  if (cnt == 0) return -1;
  NdNode nd;
  nd.x0 = x0; nd.y0 = y0; nd.x1 = x1; nd.y1 = y1;
  if (cnt <= kLeaf || (x1 - x0 <= 1 && y1 - y0 <= 1)) {
    for (int j = y0; j < y1; ++j)
      for (int i = x0; i < x1; ++i)
        if (cls[int64_t(j) * g.nx + i] == 1) nd.sep.push_back(int64_t(j) * g.nx + i);
  } else if (x1 - x0 >= y1 - y0) {
    const int xs = (x0 + x1) / 2;
    nd.child[0] = nd_build(t, g, cls, x0, y0, xs, y1);
    nd.child[1] = nd_build(t, g, cls, xs + 1, y0, x1, y1);
    for (int j = y0; j < y1; ++j)
      if (cls[int64_t(j) * g.nx + xs] == 1) nd.sep.push_back(int64_t(j) * g.nx + xs);
  } else {
    const int ys = (y0 + y1) / 2;
    nd.child[0] = nd_build(t, g, cls, x0, y0, x1, ys);
    nd.child[1] = nd_build(t, g, cls, x0, ys + 1, x1, y1);
    for (int i = x0; i < x1; ++i)
      if (cls[int64_t(ys) * g.nx + i] == 1) nd.sep.push_back(int64_t(ys) * g.nx + i);
  }
  t.push_back(std::move(nd));
  return int(t.size()) - 1;
}

// Boundary of a tree node: the present neighbours of its members that are
// not members (class-1 nodes outside the box, or kept nodes), sorted.
void nd_boundary(const Grid& g, const std::vector<uint8_t>& cls, const NdNode& X,
                 std::vector<int>& stamp, int sid, std::vector<int64_t>& out) {
  out.clear();
  for (int j = X.y0; j < X.y1; ++j)
    for (int i = X.x0; i < X.x1; ++i) {
      const int64_t n = int64_t(j) * g.nx + i;
      if (cls[n] != 1) continue;
      const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
      for (int q = 0; q < 4; ++q) {
        const int ii = i + di[q], jj = j + dj[q];
        if (ii < 0 || jj < 0 || ii >= g.nx || jj >= g.ny) continue;
        const int64_t nn = int64_t(jj) * g.nx + ii;
        const uint8_t c = cls[nn];
        if (c == 0) continue;
        const bool inside = ii >= X.x0 && ii < X.x1 && jj >= X.y0 && jj < X.y1;
        if (c == 1 && inside) continue;
        if (stamp[nn] != sid) {
          stamp[nn] = sid;
          out.push_back(nn);
        }
      }
    }
  std::sort(out.begin(), out.end());
}

// Schur update on an index list (grid ids, then the two extra columns as ids
// N and N+1), lower triangle m x m.
struct Update {
  std::vector<int64_t> idx;
  std::vector<cd> U;
};

// Stage 1: eliminate every class-1 node of the augmented operator [A f w]
// by multifrontal nested dissection; returns the Schur update on (kept nodes
// adjacent to the eliminated ones, f, w).
int exterior_schur(const Grid& g, const std::vector<uint8_t>& cls, const Operator& op,
                   const std::vector<cd>& f, const std::vector<cd>& w, int nt, Update* out) {
  const int64_t N = int64_t(g.nx) * g.ny;
  std::vector<NdNode> t;
  const int root = nd_build(t, g, cls, 0, 0, g.nx, g.ny);
  if (root < 0) {
    out->idx = {N, N + 1};
    out->U.assign(4, cd(0.0));
    return PNGF_OK;
  }
  std::vector<Update> upd(t.size());
  std::vector<int> stamp(N + 2, -1), mark(N + 2, -1), pos(N + 2, -1);
  std::vector<int64_t> bnd, idx;
  std::vector<cd> F;
  for (int x = 0; x < int(t.size()); ++x) {
    const NdNode& X = t[x];
    nd_boundary(g, cls, X, stamp, x, bnd);
    idx = bnd;
    idx.push_back(N);
    idx.push_back(N + 1);
    const int nb = int(idx.size());
    idx.insert(idx.end(), X.sep.begin(), X.sep.end());
    const int m = int(idx.size());
    for (int p = 0; p < m; ++p) {
      mark[idx[p]] = x;
      pos[idx[p]] = p;
    }
    F.assign(size_t(m) * m, cd(0.0));
    auto at = [&](int r, int c) -> cd& {
      return F[size_t(std::max(r, c)) * m + std::min(r, c)];
    };
    // original entries of the separator's rows (pairs inside the separator
    // once; pairs with a boundary node here, pairs with an already
    // eliminated node were taken by that node's front)
    for (int64_t n : X.sep) {
      const int pn = pos[n];
      at(pn, pn) += op.diag[n];
      at(pn, nb - 2) += f[n];
      at(pn, nb - 1) += w[n];
      const int i = int(n % g.nx), j = int(n / g.nx);
      const int64_t nbr[4] = {i > 0 ? n - 1 : -1, i + 1 < g.nx ? n + 1 : -1,
                              j > 0 ? n - g.nx : -1, j + 1 < g.ny ? n + g.nx : -1};
      for (int64_t nn : nbr) {
        if (nn < 0 || mark[nn] != x) continue;
        const int pm = pos[nn];
        if (pm >= nb && nn < n) continue;  // both in the separator: once
        at(pn, pm) += link(op, n, nn);
      }
    }
    for (int c : X.child) {
      if (c < 0) continue;
      Update& u = upd[c];
      const int mc = int(u.idx.size());
      std::vector<int> pc(mc);
      for (int r = 0; r < mc; ++r) {
        if (mark[u.idx[r]] != x) return PNGF_EINVAL;  // not nested: a bug, never data
        pc[r] = pos[u.idx[r]];
      }
      for (int r = 0; r < mc; ++r)
        for (int q = 0; q <= r; ++q) at(pc[r], pc[q]) += u.U[size_t(r) * mc + q];
      std::vector<int64_t>().swap(u.idx);
      std::vector<cd>().swap(u.U);
    }
    const int st = eliminate_last(F.data(), m, m, m - nb, false, nt);
    if (st != PNGF_OK) return st;
    Update& u = upd[x];
    u.idx.assign(idx.begin(), idx.begin() + nb);
    u.U.resize(size_t(nb) * nb);
    for (int r = 0; r < nb; ++r)
      std::memcpy(&u.U[size_t(r) * nb], &F[size_t(r) * m], sizeof(cd) * (r + 1));
  }
  *out = std::move(upd[root]);
  return PNGF_OK;
}

// Stage 2: G = -(S_D)^-1 for the design pixels, S_D assembled from the
// operator on D and the root update of stage 1.  Also returns r_D, v and c.
int design_inverse(const Grid& g, const std::vector<int64_t>& dnodes,
                   const std::vector<int>& pix_of, const Operator& op, const Update& ext,
                   const std::vector<cd>& f, const std::vector<cd>& w, int nt,
                   std::vector<cd>& G, std::vector<cd>& rd, std::vector<cd>& v, cd* c) {
  const int64_t N = int64_t(g.nx) * g.ny;
  const int n = int(dnodes.size());
  // class 1: interior pixels (all four neighbours are pixels); class 2: the
  // perimeter, which the exterior couples densely
  std::vector<uint8_t> cls(N, 0);
  int x0 = g.nx, y0 = g.ny, x1 = 0, y1 = 0;
  for (int64_t q : dnodes) {
    const int i = int(q % g.nx), j = int(q / g.nx);
    const bool inner = pix_of[q - 1] >= 0 && pix_of[q + 1] >= 0 && pix_of[q - g.nx] >= 0 &&
                       pix_of[q + g.nx] >= 0;
    cls[q] = inner ? 1 : 2;
    x0 = std::min(x0, i); x1 = std::max(x1, i + 1);
    y0 = std::min(y0, j); y1 = std::max(y1, j + 1);
  }
  std::vector<NdNode> t;
  nd_build(t, g, cls, x0, y0, x1, y1);
  // ordering: the separators in postorder, then the perimeter
  std::vector<int> posq(n, -1), lo(t.size()), hi(t.size());
  std::vector<int> ord;  // position -> pixel
  ord.reserve(n);
  for (int x = 0; x < int(t.size()); ++x) {
    const NdNode& X = t[x];
    int start = int(ord.size());
    if (X.child[0] >= 0) start = lo[X.child[0]];
    else if (X.child[1] >= 0) start = lo[X.child[1]];
    lo[x] = start;
    for (int64_t nd : X.sep) {
      posq[pix_of[nd]] = int(ord.size());
      ord.push_back(pix_of[nd]);
    }
    hi[x] = int(ord.size());
  }
  const int n_in = int(ord.size());
  for (int q = 0; q < n; ++q)
    if (cls[dnodes[q]] == 2) {
      posq[q] = int(ord.size());
      ord.push_back(q);
    }
  if (int(ord.size()) != n) return PNGF_EINVAL;
  const int n_per = n - n_in;

  // S_D in the new order (lower triangle of W)
  std::vector<cd> W(size_t(n) * n, cd(0.0));
  auto at = [&](int r, int cc) -> cd& {
    return W[size_t(std::max(r, cc)) * n + std::min(r, cc)];
  };
  rd.assign(n, 0.0);
  v.assign(n, 0.0);
  for (int q = 0; q < n; ++q) {
    const int64_t nd = dnodes[q];
    at(posq[q], posq[q]) += op.diag[nd];
    rd[q] = f[nd];
    v[q] = w[nd];
    int qq;
    if ((qq = pix_of[nd + 1]) >= 0) at(posq[q], posq[qq]) += op.xl[nd];
    if ((qq = pix_of[nd + g.nx]) >= 0) at(posq[q], posq[qq]) += op.yl[nd];
  }
  const int me = int(ext.idx.size());
  std::vector<int> pe(me, -1);  // pixel id, or -1 / -2 for f / w
  for (int r = 0; r < me; ++r) {
    const int64_t id = ext.idx[r];
    if (id == N) pe[r] = -1;
    else if (id == N + 1) pe[r] = -2;
    else {
      if (id < 0 || id >= N || pix_of[id] < 0) return PNGF_EINVAL;
      pe[r] = pix_of[id];
    }
  }
  *c = 0.0;
  for (int r = 0; r < me; ++r)
    for (int q = 0; q <= r; ++q) {
      const cd u = ext.U[size_t(r) * me + q];
      const int a = pe[r], b = pe[q];
      if (a >= 0 && b >= 0) at(posq[a], posq[b]) += u;
      else if (a >= 0) (b == -1 ? rd[a] : v[a]) += u;
      else if (b >= 0) (a == -1 ? rd[b] : v[b]) += u;
      else if (a != b) *c = -u;  // the (w, f) entry is -w_O^T A_OO^-1 f_O
    }

  // sweeps of the interior separators, each on the rows it couples to
  std::vector<int> stamp(N, -1);
  std::vector<int64_t> bnd;
  std::vector<int> R;
  std::vector<cd> Wg;
  for (int x = 0; x < int(t.size()); ++x) {
    const NdNode& X = t[x];
    const int b = int(X.sep.size());
    nd_boundary(g, cls, X, stamp, x, bnd);
    R.clear();
    for (int p = lo[x]; p < hi[x] - b; ++p) R.push_back(p);
    for (int64_t nd : bnd) R.push_back(posq[pix_of[nd]]);
    for (int p = hi[x] - b; p < hi[x]; ++p) R.push_back(p);
    const int m = int(R.size());
    Wg.resize(size_t(m) * m);
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt) if (nt > 1 && m > 512)
    for (int r = 0; r < m; ++r)
      for (int q = 0; q <= r; ++q) Wg[size_t(r) * m + q] = at(R[r], R[q]);
    const int st = eliminate_last(Wg.data(), m, m, b, true, nt);
    if (st != PNGF_OK) return st;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt) if (nt > 1 && m > 512)
    for (int r = 0; r < m; ++r)
      for (int q = 0; q <= r; ++q) at(R[r], R[q]) = Wg[size_t(r) * m + q];
  }
  std::vector<cd>().swap(Wg);
  // the perimeter couples to everything: one sweep of the whole matrix
  int st = eliminate_last(W.data(), n, n, n_per, true, nt);
  if (st != PNGF_OK) return st;

  G.resize(size_t(n) * n);
#pragma omp parallel for schedule(static) num_threads(nt) if (nt > 1)
  for (int a = 0; a < n; ++a) {
    const int pa = posq[a];
    cd* Ga = &G[size_t(a) * n];
    for (int b = 0; b < n; ++b) {
      const int pb = posq[b];
      Ga[b] = W[size_t(std::max(pa, pb)) * n + std::min(pa, pb)];
    }
  }
  return PNGF_OK;
}

}  // namespace

int dense_inverse(cd* a, int n, int ld) { return gj_inverse(a, n, ld, omp_get_max_threads()); }

int precompute(const pngf_problem* p, Precomputed* out, std::string* err) {
  auto t0 = std::chrono::steady_clock::now();
  if (!p || !out) { *err = "null argument"; return PNGF_EINVAL; }
  if (p->nx < 3 || p->ny < 3 || p->npml < 0 || !(p->h > 0.0)) {
    *err = "bad grid sizes";
    return PNGF_EINVAL;
  }
  if (!p->eps_static || !p->design_mask || !p->k0 || !p->src || !p->w) {
    *err = "null problem array";
    return PNGF_EINVAL;
  }
  if (p->nfreq < 1 || p->nobj != 1) {
    *err = "need nfreq >= 1 and nobj == 1";
    return PNGF_EINVAL;
  }
  if (p->pixel_kind != PNGF_PIXEL_DIELECTRIC && p->pixel_kind != PNGF_PIXEL_PEC) {
    *err = "unknown pixel_kind";
    return PNGF_EINVAL;
  }
  if (p->objective_kind < PNGF_POINT_INTENSITY || p->objective_kind > PNGF_MEAN_TRANSMISSION) {
    *err = "unknown objective_kind";
    return PNGF_EINVAL;
  }
  Grid g{p->nx, p->ny, p->npml, p->h};
  const int64_t N = int64_t(g.nx) * g.ny;
  out->grid = g;
  out->eps_lo = p->eps_lo;
  out->eps_hi = p->eps_hi;
  out->pec = p->pixel_kind == PNGF_PIXEL_PEC;
  out->design_nodes.clear();
  std::vector<int> pix_of(N, -1);
  for (int64_t n = 0; n < N; ++n) {
    if (!p->design_mask[n]) continue;
    int i = int(n % g.nx), j = int(n / g.nx);
    if (i < g.npml + 1 || i > g.nx - 2 - g.npml || j < g.npml + 1 || j > g.ny - 2 - g.npml) {
      *err = "design pixel inside the PML or on the grid edge";
      return PNGF_EINVAL;
    }
    pix_of[n] = int(out->design_nodes.size());
    out->design_nodes.push_back(n);
  }
  const int nd = int(out->design_nodes.size());
  if (nd < 1) { *err = "empty design region"; return PNGF_EINVAL; }
  out->n_d = nd;

  std::vector<double> eps(p->eps_static, p->eps_static + N);
  for (int64_t n : out->design_nodes) eps[n] = p->eps_lo;
  std::vector<uint8_t> cls_ext(N, 1);
  for (int64_t n : out->design_nodes) cls_ext[n] = 2;
  const bool norm_hom = p->objective_kind == PNGF_MEAN_TRANSMISSION;

  out->freq.assign(p->nfreq, FreqData());
  // frequencies run concurrently; the threads left over go to each
  // frequency's dense kernels
  const int T = std::max(1, omp_get_max_threads());
  const int outer = std::min(p->nfreq, T);
  const int inner = std::max(1, T / outer);
  const int saved_levels = omp_get_max_active_levels();
  omp_set_max_active_levels(2);
  std::vector<int> status(p->nfreq, PNGF_OK);
  std::vector<std::string> msgs(p->nfreq);
#pragma omp parallel for schedule(dynamic, 1) num_threads(outer)
  for (int fi = 0; fi < p->nfreq; ++fi) {
    FreqData& F = out->freq[fi];
    const double k0 = p->k0[fi];
    F.k0 = k0;
    F.norm = p->obj_norm ? p->obj_norm[fi] : 1.0;
    Operator op = build_operator(g, eps, k0);
    // scaled right-hand side f = S i k0 J and the output functional w
    const double* J = p->src + size_t(fi) * 2 * N;
    std::vector<cd> f(N), w(N);
    for (int64_t n = 0; n < N; ++n) {
      f[n] = op.scale[n] * cd(0.0, k0) * cd(J[2 * n], J[2 * n + 1]);
      w[n] = cd(p->w[2 * n], p->w[2 * n + 1]);
    }
    Update ext;
    int st = exterior_schur(g, cls_ext, op, f, w, inner, &ext);
    if (st != PNGF_OK) {
      status[fi] = st;
      msgs[fi] = "singular pivot block in the exterior elimination";
      continue;
    }
    std::vector<cd> rd, v;
    cd c = 0.0;
    st = design_inverse(g, out->design_nodes, pix_of, op, ext, f, w, inner, F.G, rd, v, &c);
    if (st != PNGF_OK) {
      status[fi] = st;
      msgs[fi] = "singular pivot block in the design-region inverse";
      continue;
    }
    // b = E_b[D] = -G r_D, G_OD = v^T G, x_b = c + v^T b
    F.b.assign(nd, 0.0);
    F.god.assign(nd, 0.0);
    for (int a = 0; a < nd; ++a) {
      cd sb = 0.0, sg = 0.0;
      const cd* Ga = &F.G[size_t(a) * nd];
      for (int q = 0; q < nd; ++q) {
        sb += Ga[q] * rd[q];
        sg += Ga[q] * v[q];
      }
      F.b[a] = -sb;
      F.god[a] = sg;
    }
    cd xb = c;
    for (int q = 0; q < nd; ++q) xb += v[q] * F.b[q];
    F.xb = xb;
    if (norm_hom) {
      // vacuum transmission of the same source and output: every node
      // eliminated, the (w, f) entry of the root update is -w^T A^-1 f
      std::vector<double> one(N, 1.0);
      Operator oh = build_operator(g, one, k0);
      for (int64_t n = 0; n < N; ++n) f[n] = oh.scale[n] * cd(0.0, k0) * cd(J[2 * n], J[2 * n + 1]);
      std::vector<uint8_t> all(N, 1);
      Update uh;
      st = exterior_schur(g, all, oh, f, w, inner, &uh);
      if (st != PNGF_OK) {
        status[fi] = st;
        msgs[fi] = "singular pivot block in the vacuum solve";
        continue;
      }
      const cd xh = -uh.U[size_t(1) * 2 + 0];
      const double t = std::norm(xh);
      if (!(t > 0.0) || !std::isfinite(t)) {
        status[fi] = PNGF_ENUMERIC;
        msgs[fi] = "zero vacuum transmission: the mean-transmission objective is undefined";
        continue;
      }
      F.norm *= t;
    }
  }
  omp_set_max_active_levels(saved_levels);
  for (int fi = 0; fi < p->nfreq; ++fi)
    if (status[fi] != PNGF_OK) {
      *err = msgs[fi];
      return status[fi];
    }
  out->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return PNGF_OK;
}

}  // namespace pngf
