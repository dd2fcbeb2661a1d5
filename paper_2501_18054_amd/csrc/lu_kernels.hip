// FP64 direct inversion of the PNGF system matrix on the GPU (gfx950).
//
// Used for the initial inverse C0^-1 = [(I - k0^2 G diag(deps))]^-1 (Direct
// binary search: the inverse of the initial system matrix is found and stored)
// and for the periodic re-inversion that bounds the drift of long chains of
// low-rank updates (Computational efficiency: direct re-inversion instead of
// Woodbury when many unknowns have changed).
//
// Method: blocked Gauss-Jordan elimination with partial pivoting, in place.
// Pivoting is virtual (rows are never moved): column k picks the unused row
// p_k with the largest |entry|, so the elimination is that of Pi A with
// (Pi A)[k,:] = A[p_k,:], and the in-place result M satisfies
// (Pi A)^-1 [k,:] = M[p_k,:].  Since A^-1 = (Pi A)^-1 Pi, the final gather is
//     A^-1[i, p_l] = M[p_i, l].
// Blocking (panel width nb): the panel columns [k0, k0+nb) are reduced by one
// workgroup (pivot search, pivot-row scaling and elimination inside the panel,
// giving [-B01 B11^-1; B11^-1; -B21 B11^-1] in place); then every column
// outside the panel is updated by the rank-nb product
//     M[r, j] = (r is a pivot of this panel ? 0 : M[r, j]) + P[r,:] B1[:, j],
// where B1 holds the panel's pivot rows before the update.  On gfx950 the
// FP64 matrix-core rate equals the FP64 vector rate (78.6 TFLOP/s), and at
// nb = 16 the update is HBM-bound, so it runs on the vector ALUs.
#include "dev_state.h"

namespace pngf {

constexpr int kGjNb = 16;
constexpr int kUpdRows = 32;

// S = I - k0^2 G diag(deps) (rows of length nd, stride ld); clears pivot marks.
__global__ __launch_bounds__(256) void k_build_system(z64* S, const z64* G, int nd, int ld,
                                                      const uint8_t* bits, double k2d,
                                                      int32_t* used) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < nd) {
    const double s = bits[j] ? -k2d : 0.0;
    z64 g = G[size_t(i) * ld + j];
    z64 v = {g.re * s + (i == j ? 1.0 : 0.0), g.im * s};
    S[size_t(i) * ld + j] = v;
  }
  if (i == 0 && j < nd) used[j] = 0;
}

// Panel columns [k0, k0+ncols) of S gathered into a contiguous n x kGjNb
// buffer (row r at Pb[r*kGjNb]) so the panel reduction streams whole rows.
__global__ __launch_bounds__(256) void k_gj_panel_in(const z64* S, int ld, int n, int k0,
                                                     int ncols, z64* Pb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int r = e / kGjNb, c = e % kGjNb;
  if (r < n) Pb[e] = (c < ncols) ? S[size_t(r) * ld + k0 + c] : z64{0.0, 0.0};
}

__global__ __launch_bounds__(256) void k_gj_panel_out(z64* S, int ld, int n, int k0, int ncols,
                                                      const z64* Pb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int r = e / kGjNb, c = e % kGjNb;
  if (r < n && c < ncols) S[size_t(r) * ld + k0 + c] = Pb[e];
}

// ---- panel by tournament pivoting ------------------------------------------
// The panel's kGjNb pivot rows are chosen by a reduction tree of partial-
// pivoting eliminations (tournament pivoting, Grigori-Demmel-Xiang CALU):
// every group of <= kTsRows candidate rows is reduced by Gaussian elimination
// with partial pivoting on its panel entries and proposes the rows it pivoted
// on; groups of proposals are reduced again until one group remains.  The
// winners B11 (kGjNb x kGjNb) are inverted, and every row is then reduced
// independently: pivot rows get B11^-1, the others -B_r B11^-1, which is the
// Gauss-Jordan panel [-B01 B11^-1; B11^-1; -B21 B11^-1].
constexpr int kTsRows = 256;      // candidate rows per group (one per thread)
constexpr int kTsFan = kTsRows / kGjNb;  // proposals merged per group

// One group per workgroup.  level0: the group is rows [g*kTsRows, ...) minus
// rows already used as pivots; otherwise the proposals of groups
// [g*kTsFan, (g+1)*kTsFan) of the previous level.  Writes the group's
// proposals (in pivot order) to out[g*kGjNb + c] and their count to cnt_out[g].
// final_: also writes piv/used and B11^-1 (row c <-> column k0+c).
__global__ __launch_bounds__(256) void k_tsel(const z64* Pb, int n, int k0, int ncols, int level0,
                                              const int32_t* in, const int32_t* cnt_in,
                                              int ngroups_in, int32_t* out, int32_t* cnt_out,
                                              int final_, int32_t* piv, int32_t* used,
                                              z64* B11inv, int32_t* status) {
  __shared__ z64 A[kTsRows][kGjNb + 1];   // +1: conflict-free LDS rows
  __shared__ int idx[kTsRows];
  __shared__ int alive[kTsRows];
  __shared__ int s_m;
  __shared__ int sel[kGjNb];
  __shared__ double s_val[256 / 64];
  __shared__ int s_idx[256 / 64];
  __shared__ z64 W[kGjNb][2 * kGjNb];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int g = blockIdx.x;
  // Slot tid holds one candidate: row g*kTsRows+tid (level 0, if not yet a
  // pivot) or proposal tid%kGjNb of group g*kTsFan+tid/kGjNb.
  {
    int row = -1;
    if (level0) {
      const int r = g * kTsRows + tid;
      if (r < n && !used[r]) row = r;
    } else {
      const int q = g * kTsFan + tid / kGjNb, t = tid % kGjNb;
      if (q < ngroups_in && t < cnt_in[q]) row = in[q * kGjNb + t];
    }
    idx[tid] = row;
    alive[tid] = row >= 0 ? 1 : 0;
    const int cnt = __syncthreads_count(row >= 0);
    if (tid == 0) s_m = cnt;
  }
  __syncthreads();
  const int m = s_m;
  for (int e = tid; e < kTsRows * kGjNb; e += 256) {
    const int i = e / kGjNb, c = e % kGjNb;
    A[i][c] = (idx[i] >= 0) ? Pb[size_t(idx[i]) * kGjNb + c] : z64{0.0, 0.0};
  }
  __syncthreads();
  const int nsel = min(ncols, m);
  for (int c = 0; c < nsel; ++c) {
    double best = -1.0;
    int bi = kTsRows;
    if (alive[tid]) { best = zabs2(A[tid][c]); bi = tid; }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { s_val[wid] = best; s_idx[wid] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = s_val[0];
      int p = s_idx[0];
      for (int w = 1; w < 4; ++w)
        if (s_val[w] > b || (s_val[w] == b && s_idx[w] < p)) { b = s_val[w]; p = s_idx[w]; }
      if (p >= kTsRows) p = 0;
      if (final_ && !(b > 0.0)) atomicOr(status, 1);
      sel[c] = p;
      alive[p] = 0;
    }
    __syncthreads();
    const int p = sel[c];
    // eliminate column c from the remaining rows of the group (c' > c only)
    if (alive[tid]) {
      const z64 piv_v = A[p][c];
      const double d = zabs2(piv_v);
      const z64 l = (d > 0.0) ? zdiv(A[tid][c], piv_v) : z64{0.0, 0.0};
      for (int cc = c + 1; cc < kGjNb; ++cc) A[tid][cc] = zsub(A[tid][cc], zmul(l, A[p][cc]));
    }
    __syncthreads();
  }
  if (tid < nsel) out[g * kGjNb + tid] = idx[sel[tid]];
  if (tid == 0) cnt_out[g] = nsel;
  if (!final_) return;
  // B11 from the untouched panel rows of the winners, inverted by Gauss-Jordan
  // in the winners' order (their elimination above needed no interchange).
  for (int e = tid; e < kGjNb * 2 * kGjNb; e += 256) {
    const int r = e / (2 * kGjNb), c = e % (2 * kGjNb);
    z64 v{0.0, 0.0};
    if (c < kGjNb) {
      if (r < nsel && c < ncols) v = Pb[size_t(idx[sel[r]]) * kGjNb + c];
      else if (r == c) v = z64{1.0, 0.0};       // padding of a ragged panel
    } else if (c - kGjNb == r) {
      v = z64{1.0, 0.0};
    }
    W[r][c] = v;
  }
  __syncthreads();
  __shared__ z64 fcol[kGjNb];
  for (int c = 0; c < kGjNb; ++c) {
    const z64 pv = W[c][c];
    const z64 inv = (zabs2(pv) > 0.0) ? zdiv(z64{1.0, 0.0}, pv) : z64{0.0, 0.0};
    __syncthreads();
    if (tid < 2 * kGjNb) W[c][tid] = zmul(W[c][tid], inv);
    if (tid < kGjNb) fcol[tid] = W[tid][c];
    __syncthreads();
    for (int e = tid; e < kGjNb * 2 * kGjNb; e += 256) {
      const int r = e / (2 * kGjNb), cc = e % (2 * kGjNb);
      if (r != c) W[r][cc] = zsub(W[r][cc], zmul(fcol[r], W[c][cc]));
    }
    __syncthreads();
  }
  for (int e = tid; e < kGjNb * kGjNb; e += 256) {
    const int r = e / kGjNb, c = e % kGjNb;
    B11inv[e] = W[r][kGjNb + c];
  }
  if (tid < nsel) {
    const int row = idx[sel[tid]];
    piv[k0 + tid] = row;
    used[row] = k0 + tid + 1;
  }
}

// Every panel row reduced by B11^-1: pivot rows (used[r]-1 in the panel) get
// their row of B11^-1, the others -B_r B11^-1.  A workgroup handles 16 rows,
// one thread per output entry.
__global__ __launch_bounds__(256) void k_tapply(z64* Pb, int n, int k0, int ncols,
                                                const int32_t* used, const z64* B11inv) {
  __shared__ z64 Bi[kGjNb][kGjNb];
  __shared__ z64 R[256 / kGjNb][kGjNb + 1];
  const int tid = threadIdx.x;
  const int rr = tid / kGjNb, cc = tid % kGjNb;
  const int r = blockIdx.x * (256 / kGjNb) + rr;
  Bi[rr][cc] = B11inv[tid];
  R[rr][cc] = (r < n) ? Pb[size_t(r) * kGjNb + cc] : z64{0.0, 0.0};
  __syncthreads();
  if (r >= n) return;
  const int u = used[r] - 1;
  z64 out;
  if (u >= k0 && u < k0 + ncols) {
    out = Bi[u - k0][cc];
  } else {
    z64 acc{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kGjNb; ++q) acc = zfma(R[rr][q], Bi[q][cc], acc);
    out = z64{-acc.re, -acc.im};
  }
  Pb[size_t(r) * kGjNb + cc] = (cc < ncols) ? out : z64{0.0, 0.0};
}

// B1[c, :] = S[piv[k0+c], :] (the panel's pivot rows before the update).
__global__ __launch_bounds__(256) void k_gj_copy_rows(const z64* S, int ld, int n, int k0,
                                                      int ncols, const int32_t* piv, z64* B1) {
  const int c = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (c < ncols && j < n) B1[size_t(c) * ld + j] = S[size_t(piv[k0 + c]) * ld + j];
}

// Rank-ncols update of every column outside the panel.
__global__ __launch_bounds__(256) void k_gj_update(z64* S, int ld, int n, int k0, int ncols,
                                                   const z64* B1, const int32_t* used,
                                                   const z64* Pb) {
  __shared__ z64 Pt[kUpdRows][kGjNb];
  __shared__ int isp[kUpdRows];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.y * kUpdRows;
  for (int e = tid; e < kUpdRows * kGjNb; e += 256) {
    const int rr = e / kGjNb, c = e % kGjNb;
    const int r = r0 + rr;
    Pt[rr][c] = (r < n && c < ncols) ? Pb[size_t(r) * kGjNb + c] : z64{0.0, 0.0};
  }
  if (tid < kUpdRows) {
    const int r = r0 + tid;
    const int u = (r < n) ? used[r] - 1 : -1;
    isp[tid] = (u >= k0 && u < k0 + ncols) ? 1 : 0;
  }
  __syncthreads();
  const int j = blockIdx.x * 256 + tid;
  if (j >= n || (j >= k0 && j < k0 + ncols)) return;
  z64 b[kGjNb];
#pragma unroll
  for (int c = 0; c < kGjNb; ++c) b[c] = (c < ncols) ? B1[size_t(c) * ld + j] : z64{0.0, 0.0};
  const int rmax = min(kUpdRows, n - r0);
  for (int rr = 0; rr < rmax; ++rr) {
    z64* dst = S + size_t(r0 + rr) * ld + j;
    z64 acc = isp[rr] ? z64{0.0, 0.0} : *dst;
#pragma unroll
    for (int c = 0; c < kGjNb; ++c) acc = zfma(Pt[rr][c], b[c], acc);
    *dst = acc;
  }
}

// inv_p[p_l] = l
__global__ __launch_bounds__(256) void k_gj_invperm(const int32_t* piv, int32_t* inv_p, int n) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l < n) inv_p[piv[l]] = l;
}

// A^-1[i, j] = M[p_i, inv_p[j]]
__global__ __launch_bounds__(256) void k_gj_finalize(const z64* M, z64* Ainv, int ld, int n,
                                                     const int32_t* piv, const int32_t* inv_p) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) Ainv[size_t(i) * ld + j] = M[size_t(piv[i]) * ld + inv_p[j]];
}

// y[i] = beta w[i] + gamma w2[i] + alpha sum_j A[i,j] d_j v[j], with
// d_j = (bits[j] ? ds : 0) when bits != nullptr, else 1.  One workgroup per
// row; y may alias w (row i reads w[i] before writing y[i]).
__global__ __launch_bounds__(kRowThreads) void k_gemv(const z64* A, int ld, int n, const z64* v,
                                                      const uint8_t* bits, double ds, z64 alpha,
                                                      z64 beta, const z64* w, double gamma,
                                                      const z64* w2, z64* y) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int i = blockIdx.x;
  const z64* a = A + size_t(i) * ld;
  z64 acc{0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += kRowThreads) {
    z64 vj = v[j];
    if (bits) vj = zscale(vj, bits[j] ? ds : 0.0);
    acc = zfma(a[j], vj, acc);
  }
  const z64 s = block_zsum(acc, red);
  if (threadIdx.x == 0) {
    z64 out = zmul(alpha, s);
    if (w) out = zfma(beta, w[i], out);
    if (w2) out = zadd(out, zscale(w2[i], gamma));
    y[i] = out;
  }
}

// x = x_b + k0^2 sum_j god[j] deps_j E[j]; writes x into the DBS state slot f
// and (on the last frequency) the objective.  One workgroup.
__global__ __launch_bounds__(kRowThreads) void k_output(ProbDev P, int f, const z64* god, z64 xb,
                                                        int last) {
  __shared__ double red[2 * (kRowThreads / 64)];
  z64 acc{0.0, 0.0};
  const double s = P.k0sq[f] * P.deps;
  for (int j = threadIdx.x; j < P.nd; j += kRowThreads)
    if (P.bits[j]) acc = zfma(god[j], zscale(P.E[f][j], s), acc);
  const z64 t = block_zsum(acc, red);
  if (threadIdx.x == 0) {
    P.st->x[f] = zadd(xb, t);
    if (last) {
      double fs = 0.0;
      for (int g = 0; g < P.nfreq; ++g) fs += P.coef[g] * zabs2(P.st->x[g]);
      P.st->f = fs;
    }
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_inverse(z64* S, z64* Cinv, const z64* G, int nd, int ld, const uint8_t* bits,
                          double k2d, z64* B1, z64* Pb, int32_t* piv, int32_t* inv_p,
                          int32_t* used, int32_t* status, int32_t* tsbuf, z64* B11inv,
                          hipStream_t s) {
  // tournament buffers: two proposal lists and two count lists
  const int g0 = (nd + kTsRows - 1) / kTsRows;
  int32_t* candA = tsbuf;
  int32_t* candB = tsbuf + g0 * kGjNb;
  int32_t* cntA = tsbuf + 2 * g0 * kGjNb;
  int32_t* cntB = cntA + g0;
  const dim3 gcols((nd + 255) / 256);
  hipLaunchKernelGGL(k_build_system, dim3(gcols.x, nd), dim3(256), 0, s, S, G, nd, ld, bits, k2d,
                     used);
  for (int k0 = 0; k0 < nd; k0 += kGjNb) {
    const int nc = min(kGjNb, nd - k0);
    const dim3 gpan((nd * kGjNb + 255) / 256);
    hipLaunchKernelGGL(k_gj_panel_in, gpan, dim3(256), 0, s, S, ld, nd, k0, nc, Pb);
    {
      int groups = g0;
      int32_t *cin = nullptr, *nin = nullptr, *cout = candA, *nout = cntA;
      int level0 = 1, ngin = 0;
      while (true) {
        const int fin = (groups == 1) ? 1 : 0;
        hipLaunchKernelGGL(k_tsel, dim3(groups), dim3(256), 0, s, Pb, nd, k0, nc, level0, cin,
                           nin, ngin, cout, nout, fin, piv, used, B11inv, status);
        if (fin) break;
        level0 = 0;
        cin = cout;
        nin = nout;
        ngin = groups;
        cout = (cout == candA) ? candB : candA;
        nout = (nout == cntA) ? cntB : cntA;
        groups = (groups + kTsFan - 1) / kTsFan;
      }
      hipLaunchKernelGGL(k_tapply, dim3((nd + 15) / 16), dim3(256), 0, s, Pb, nd, k0, nc, used,
                         B11inv);
    }
    hipLaunchKernelGGL(k_gj_copy_rows, dim3(gcols.x, nc), dim3(256), 0, s, S, ld, nd, k0, nc,
                       piv, B1);
    hipLaunchKernelGGL(k_gj_update, dim3(gcols.x, (nd + kUpdRows - 1) / kUpdRows), dim3(256), 0,
                       s, S, ld, nd, k0, nc, B1, used, Pb);
    hipLaunchKernelGGL(k_gj_panel_out, gpan, dim3(256), 0, s, S, ld, nd, k0, nc, Pb);
  }
  hipLaunchKernelGGL(k_gj_invperm, dim3(gcols.x), dim3(256), 0, s, piv, inv_p, nd);
  hipLaunchKernelGGL(k_gj_finalize, dim3(gcols.x, nd), dim3(256), 0, s, S, Cinv, ld, nd, piv,
                     inv_p);
  return hipGetLastError();
}

hipError_t launch_gemv(const z64* A, int ld, int n, const z64* v, const uint8_t* bits, double ds,
                       z64 alpha, z64 beta, const z64* w, double gamma, const z64* w2, z64* y,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3(n), dim3(kRowThreads), 0, s, A, ld, n, v, bits, ds, alpha, beta,
                     w, gamma, w2, y);
  return hipGetLastError();
}

hipError_t launch_output(const ProbDev& P, int f, const z64* god, z64 xb, int last,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(1), dim3(kRowThreads), 0, s, P, f, god, xb, last);
  return hipGetLastError();
}

}  // namespace pngf
