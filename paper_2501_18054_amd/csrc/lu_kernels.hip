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

constexpr int kPanelThreads = 1024;
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

// Panel reduction of columns [k0, k0+ncols) by one workgroup.
// used[r] = k+1 once row r is the pivot of column k.
__global__ __launch_bounds__(kPanelThreads) void k_gj_panel(z64* S, int ld, int n, int k0,
                                                            int ncols, int32_t* piv,
                                                            int32_t* used, int32_t* status) {
  __shared__ double s_val[kPanelThreads / 64];
  __shared__ int s_idx[kPanelThreads / 64];
  __shared__ z64 prow[kGjNb];
  __shared__ int s_p;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = 0; c < ncols; ++c) {
    const int k = k0 + c;
    double best = -1.0;
    int bi = n;
    for (int r = tid; r < n; r += kPanelThreads) {
      if (used[r]) continue;
      const double a = zabs2(S[size_t(r) * ld + k]);
      if (a > best) { best = a; bi = r; }
    }
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
      for (int w = 1; w < kPanelThreads / 64; ++w)
        if (s_val[w] > b || (s_val[w] == b && s_idx[w] < p)) { b = s_val[w]; p = s_idx[w]; }
      if (!(b > 0.0) || p >= n) {
        atomicOr(status, 1);
        p = (p >= n) ? 0 : p;
      }
      used[p] = k + 1;
      piv[k] = p;
      s_p = p;
    }
    __syncthreads();
    const int p = s_p;
    if (tid < ncols) {
      const z64 pv = S[size_t(p) * ld + k];
      const z64 inv = zdiv(z64{1.0, 0.0}, pv);
      const z64 v = S[size_t(p) * ld + k0 + tid];
      prow[tid] = (tid == c) ? inv : zmul(v, inv);
    }
    __syncthreads();
    if (tid < ncols) S[size_t(p) * ld + k0 + tid] = prow[tid];
    for (int r = tid; r < n; r += kPanelThreads) {
      if (r == p) continue;
      z64* row = S + size_t(r) * ld + k0;
      const z64 f = row[c];
      if (f.re == 0.0 && f.im == 0.0) continue;
      for (int cc = 0; cc < ncols; ++cc) {
        const z64 base = (cc == c) ? z64{0.0, 0.0} : row[cc];
        row[cc] = zsub(base, zmul(f, prow[cc]));
      }
    }
    __syncthreads();
  }
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
                                                   const z64* B1, const int32_t* used) {
  __shared__ z64 Pt[kUpdRows][kGjNb];
  __shared__ int isp[kUpdRows];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.y * kUpdRows;
  for (int e = tid; e < kUpdRows * kGjNb; e += 256) {
    const int rr = e / kGjNb, c = e % kGjNb;
    const int r = r0 + rr;
    Pt[rr][c] = (r < n && c < ncols) ? S[size_t(r) * ld + k0 + c] : z64{0.0, 0.0};
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
                          double k2d, z64* B1, int32_t* piv, int32_t* inv_p, int32_t* used,
                          int32_t* status, hipStream_t s) {
  const dim3 gcols((nd + 255) / 256);
  hipLaunchKernelGGL(k_build_system, dim3(gcols.x, nd), dim3(256), 0, s, S, G, nd, ld, bits, k2d,
                     used);
  for (int k0 = 0; k0 < nd; k0 += kGjNb) {
    const int nc = min(kGjNb, nd - k0);
    hipLaunchKernelGGL(k_gj_panel, dim3(1), dim3(kPanelThreads), 0, s, S, ld, nd, k0, nc, piv,
                       used, status);
    hipLaunchKernelGGL(k_gj_copy_rows, dim3(gcols.x, nc), dim3(256), 0, s, S, ld, nd, k0, nc,
                       piv, B1);
    hipLaunchKernelGGL(k_gj_update, dim3(gcols.x, (nd + kUpdRows - 1) / kUpdRows), dim3(256), 0,
                       s, S, ld, nd, k0, nc, B1, used);
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
