// Host precompute of libpngf (FP64, OpenMP): the once-only folding of the
// static environment into the design-region Green function.
//
// Results, Precomputation: G = B^T A^-1 B over the optimization region is the
// negated Schur complement of the augmented system [[A, B], [B^T, 0]]; the
// paper obtains it with a partial factorization (APF).  Here the same idea is
// applied to the 2D TM FDFD operator directly:
//
//   * A = S L is the complex-symmetric, PML-scaled 5-point operator
//     (S = diag(s_x s_y), which is 1 away from the PML).
//   * Order the unknowns as O (outside the design region) and D.  Then
//     (A^-1)[D,D] = (A_DD - A_DO A_OO^-1 A_OD)^-1, and A_OD only couples the
//     ring of exterior nodes that touch D to the design perimeter.
//   * A_OO is factored once by a band LDL^T (natural ordering, bandwidth nx),
//     the ring unit vectors, the exterior source and the exterior output
//     functional are forward-substituted, and every bilinear form
//     u^T A_OO^-1 v needed below is (L^-1 u)^T D^-1 (L^-1 v).
//   * The Schur complement on D is dense (N_d x N_d) and is inverted by
//     Gauss-Jordan elimination with partial pivoting:
//        G   = -(Schur)^-1                 (symmetrized; G = G^T exactly),
//        b   = E_b[D] = -G (f_D - C^T z_f),
//        G_OD = (w_D - C^T m_w)^T G,
//        x_b = w_O^T A_OO^-1 f_O - m_w^T C b + w_D^T b,
//     with f = S i k0 J, z_f = (A_OO^-1 f_O)[ring], m_w = (A_OO^-1 w_O)[ring]
//     and C the ring-to-perimeter couplings.
//
// The discrete problem (the same one the CPU oracle states independently):
//   d(u) = max(0, npml-u, u-(N-1-npml))/npml, sigma = sigma_max d^3,
//   sigma_max = -(3+1) ln(1e-8) / (2 npml h), s(u) = 1 - i sigma(u)/k0,
//   L E = [D_x (1/s_x) D_x / s_x + D_y (1/s_y) D_y / s_y + k0^2 eps] E = i k0 J,
//   Ez = 0 beyond the grid.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

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

// Band LDL^T (no pivoting) of a complex-symmetric matrix with lower bandwidth
// bw.  band[k*(bw+1) + t] holds A(k+t, k) on entry and L(k+t, k) (t > 0) /
// D(k) (t = 0) on exit.  Blocked by kLdlNb columns: a block is factored
// serially with its updates confined to the block, then the columns the block
// reaches (up to bw beyond it) receive the deferred rank-kLdlNb update in
// parallel, one OpenMP region per block.
constexpr int kLdlNb = 32;

int band_ldlt(std::vector<cd>& band, int64_t N, int bw) {
  const int W = bw + 1;
  std::vector<cd> a(W);
  for (int64_t k0 = 0; k0 < N; k0 += kLdlNb) {
    const int64_t kend = std::min<int64_t>(N, k0 + kLdlNb);
    for (int64_t k = k0; k < kend; ++k) {
      const cd d = band[k * W];
      if (std::abs(d) == 0.0 || !std::isfinite(d.real()) || !std::isfinite(d.imag()))
        return PNGF_ESINGULAR;
      const cd inv = 1.0 / d;
      const int tmax = int(std::min<int64_t>(bw, N - 1 - k));
      for (int t = 1; t <= tmax; ++t) {
        a[t] = band[k * W + t];
        band[k * W + t] = a[t] * inv;
      }
      const int tin = int(std::min<int64_t>(tmax, kend - 1 - k));
      for (int t = 1; t <= tin; ++t) {
        const cd at = a[t];
        if (at == cd(0.0, 0.0)) continue;
        cd* col = &band[(k + t) * W];
        const cd* lk = &band[k * W];
        for (int t2 = t; t2 <= tmax; ++t2) col[t2 - t] -= lk[t2] * at;
      }
    }
    const int64_t jmax = std::min<int64_t>(N, kend + bw);
#pragma omp parallel for schedule(static)
    for (int64_t j = kend; j < jmax; ++j) {
      cd* col = &band[j * W];
      for (int64_t c = std::max<int64_t>(k0, j - bw); c < kend; ++c) {
        const cd* Lc = &band[c * W];
        const cd ld = Lc[j - c] * Lc[0];
        if (ld == cd(0.0, 0.0)) continue;
        const int64_t imax = std::min<int64_t>(c + bw, N - 1);
        const double lr = ld.real(), li = ld.imag();
        double* out = reinterpret_cast<double*>(col);
        const double* lc = reinterpret_cast<const double*>(Lc);
        for (int64_t i = j; i <= imax; ++i) {
          const double xr = lc[2 * (i - c)], xi = lc[2 * (i - c) + 1];
          out[2 * (i - j)] -= xr * lr - xi * li;
          out[2 * (i - j) + 1] -= xr * li + xi * lr;
        }
      }
    }
  }
  return PNGF_OK;
}

// Y <- L^-1 Y for the unit lower band factor; Y is N x K row-major.
void band_forward(const std::vector<cd>& band, int64_t N, int bw, std::vector<cd>& Y,
                  int K, const std::vector<int64_t>& first_nz) {
  const int W = bw + 1;
  int nthreads = omp_get_max_threads();
  int chunk = std::max(1, (K + nthreads - 1) / nthreads);
#pragma omp parallel for schedule(static, 1)
  for (int c0 = 0; c0 < K; c0 += chunk) {
    const int c1 = std::min(K, c0 + chunk);
    int64_t kstart = N;
    for (int c = c0; c < c1; ++c) kstart = std::min(kstart, first_nz[c]);
    for (int64_t k = kstart; k < N; ++k) {
      const cd* yk = &Y[k * K];
      bool any = false;
      for (int c = c0; c < c1; ++c)
        if (yk[c] != cd(0.0, 0.0)) { any = true; break; }
      if (!any) continue;
      const int tmax = int(std::min<int64_t>(bw, N - 1 - k));
      for (int t = 1; t <= tmax; ++t) {
        const cd lt = band[k * W + t];
        if (lt == cd(0.0, 0.0)) continue;
        cd* yt = &Y[(k + t) * K];
        for (int c = c0; c < c1; ++c) yt[c] -= lt * yk[c];
      }
    }
  }
}

}  // namespace

int dense_inverse(cd* a, int n, int ld) {
  std::vector<int> piv(n);
  int status = PNGF_OK;
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
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      cd* ai = &a[int64_t(i) * ld];
      const cd f = ai[k];
      if (f == cd(0.0, 0.0)) continue;
      ai[k] = 0.0;
      const double fr = f.real(), fi = f.imag();
      const double* rk = reinterpret_cast<const double*>(rowk.data());
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
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) std::swap(a[int64_t(i) * ld + k], a[int64_t(i) * ld + p]);
  }
  return status;
}

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

  // Ring: exterior nodes adjacent to the design, with their couplings.
  struct Link { int ring; int pix; bool xdir; int64_t lo; };  // lo = lower node of the link
  std::vector<int64_t> ring_nodes;
  std::unordered_map<int64_t, int> ring_id;
  std::vector<Link> links;
  auto add_link = [&](int64_t o, int pix, bool xdir, int64_t lo) {
    auto it = ring_id.find(o);
    int r;
    if (it == ring_id.end()) {
      r = int(ring_nodes.size());
      ring_id.emplace(o, r);
      ring_nodes.push_back(o);
    } else {
      r = it->second;
    }
    links.push_back({r, pix, xdir, lo});
  };
  for (int q = 0; q < nd; ++q) {
    int64_t n = out->design_nodes[q];
    if (pix_of[n - 1] < 0) add_link(n - 1, q, true, n - 1);
    if (pix_of[n + 1] < 0) add_link(n + 1, q, true, n);
    if (pix_of[n - g.nx] < 0) add_link(n - g.nx, q, false, n - g.nx);
    if (pix_of[n + g.nx] < 0) add_link(n + g.nx, q, false, n);
  }
  const int nr = int(ring_nodes.size());
  const int K = nr + 2;  // ring unit vectors, exterior source, exterior output

  out->freq.assign(p->nfreq, FreqData());
  const int bw = g.nx;
  const int W = bw + 1;
  for (int fi = 0; fi < p->nfreq; ++fi) {
    FreqData& F = out->freq[fi];
    const double k0 = p->k0[fi];
    F.k0 = k0;
    F.norm = p->obj_norm ? p->obj_norm[fi] : 1.0;
    Operator op = build_operator(g, eps, k0);

    // Exterior operator A_OO in band form (design nodes decoupled, unit diag).
    std::vector<cd> band(size_t(N) * W, cd(0.0, 0.0));
    for (int64_t n = 0; n < N; ++n) {
      const bool dn = pix_of[n] >= 0;
      band[n * W] = dn ? cd(1.0, 0.0) : op.diag[n];
      if (!dn && n + 1 < N && pix_of[n + 1] < 0) band[n * W + 1] = op.xl[n];
      if (!dn && n + g.nx < N && pix_of[n + g.nx] < 0) band[n * W + g.nx] = op.yl[n];
    }
    int st = band_ldlt(band, N, bw);
    if (st != PNGF_OK) { *err = "zero pivot in the exterior band factorization"; return st; }

    // Scaled right-hand side f = S i k0 J and the output functional w.
    const double* J = p->src + size_t(fi) * 2 * N;
    std::vector<cd> f(N), w(N);
    for (int64_t n = 0; n < N; ++n) {
      f[n] = op.scale[n] * cd(0.0, k0) * cd(J[2 * n], J[2 * n + 1]);
      w[n] = cd(p->w[2 * n], p->w[2 * n + 1]);
    }
    std::vector<cd> Y(size_t(N) * K, cd(0.0, 0.0));
    std::vector<int64_t> first(K, N);
    for (int r = 0; r < nr; ++r) {
      Y[ring_nodes[r] * K + r] = 1.0;
      first[r] = ring_nodes[r];
    }
    for (int64_t n = 0; n < N; ++n) {
      if (pix_of[n] >= 0) continue;
      Y[n * K + nr] = f[n];
      Y[n * K + nr + 1] = w[n];
      if (f[n] != cd(0.0, 0.0)) first[nr] = std::min(first[nr], n);
      if (w[n] != cd(0.0, 0.0)) first[nr + 1] = std::min(first[nr + 1], n);
    }
    band_forward(band, N, bw, Y, K, first);

    // M = Y^T D^-1 Y (K x K), accumulated per thread; the partial sums are
    // added in thread order afterwards, so the result does not depend on
    // which thread finishes first.
    std::vector<cd> M(size_t(K) * K, cd(0.0, 0.0));
    const int nth = omp_get_max_threads();
    std::vector<std::vector<cd>> parts(static_cast<size_t>(nth));
#pragma omp parallel num_threads(nth)
    {
      std::vector<cd>& Ml = parts[size_t(omp_get_thread_num())];
      Ml.assign(size_t(K) * K, cd(0.0, 0.0));
#pragma omp for schedule(static)
      for (int64_t k = 0; k < N; ++k) {
        const cd* yk = &Y[k * K];
        const cd dinv = 1.0 / band[k * W];
        for (int a = 0; a < K; ++a) {
          if (yk[a] == cd(0.0, 0.0)) continue;
          const cd ya = yk[a] * dinv;
          cd* mr = &Ml[size_t(a) * K];
          for (int c = 0; c < K; ++c) mr[c] += ya * yk[c];
        }
      }
    }
    for (const std::vector<cd>& Ml : parts)
      for (size_t q = 0; q < Ml.size(); ++q) M[q] += Ml[q];
    std::vector<std::vector<cd>>().swap(parts);
    std::vector<cd>().swap(Y);
    std::vector<cd>().swap(band);

    // Schur complement on D: A_DD - C^T Z C (dense, row-major n_d x n_d).
    std::vector<cd> S(size_t(nd) * nd, cd(0.0, 0.0));
    for (int q = 0; q < nd; ++q) {
      int64_t n = out->design_nodes[q];
      S[size_t(q) * nd + q] = op.diag[n];
      int qq;
      if ((qq = pix_of[n + 1]) >= 0) { S[size_t(q) * nd + qq] = op.xl[n]; S[size_t(qq) * nd + q] = op.xl[n]; }
      if ((qq = pix_of[n + g.nx]) >= 0) { S[size_t(q) * nd + qq] = op.yl[n]; S[size_t(qq) * nd + q] = op.yl[n]; }
    }
    std::vector<cd> cval(links.size());
    for (size_t a = 0; a < links.size(); ++a)
      cval[a] = links[a].xdir ? op.xl[links[a].lo] : op.yl[links[a].lo];
    for (size_t a = 0; a < links.size(); ++a)
      for (size_t c = 0; c < links.size(); ++c)
        S[size_t(links[a].pix) * nd + links[c].pix] -=
            cval[a] * M[size_t(links[a].ring) * K + links[c].ring] * cval[c];

    st = dense_inverse(S.data(), nd, nd);
    if (st != PNGF_OK) { *err = "singular Schur complement"; return st; }
    F.G.assign(size_t(nd) * nd, 0.0);
    for (int a = 0; a < nd; ++a)
      for (int c = 0; c < nd; ++c)
        F.G[size_t(a) * nd + c] = -0.5 * (S[size_t(a) * nd + c] + S[size_t(c) * nd + a]);

    // rhs_D = f_D - C^T z_f and v = w_D - C^T m_w
    std::vector<cd> rd(nd), v(nd);
    for (int q = 0; q < nd; ++q) {
      rd[q] = f[out->design_nodes[q]];
      v[q] = w[out->design_nodes[q]];
    }
    for (size_t a = 0; a < links.size(); ++a) {
      rd[links[a].pix] -= cval[a] * M[size_t(links[a].ring) * K + nr];
      v[links[a].pix] -= cval[a] * M[size_t(links[a].ring) * K + nr + 1];
    }
    F.b.assign(nd, 0.0);
    F.god.assign(nd, 0.0);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < nd; ++a) {
      cd sb = 0.0, sg = 0.0;
      const cd* Ga = &F.G[size_t(a) * nd];
      for (int c = 0; c < nd; ++c) {
        sb += Ga[c] * rd[c];
        sg += v[c] * F.G[size_t(c) * nd + a];
      }
      F.b[a] = -sb;
      F.god[a] = sg;
    }
    cd xb = M[size_t(nr + 1) * K + nr];
    for (size_t a = 0; a < links.size(); ++a)
      xb -= M[size_t(nr + 1) * K + links[a].ring] * cval[a] * F.b[links[a].pix];
    for (int q = 0; q < nd; ++q) xb += w[out->design_nodes[q]] * F.b[q];
    F.xb = xb;
  }
  out->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return PNGF_OK;
}

}  // namespace pngf
