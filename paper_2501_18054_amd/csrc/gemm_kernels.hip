// Complex FP64 GEMM on the gfx950 matrix cores, and the small kernels of the
// FP64 block-Woodbury refresh of C^-1.
//
// GEMM: C = beta C + alpha A B with A (M x K, row-major, optionally with
// gathered columns A[i][k] = A'[i][ca[k]]) and B either K x N row-major
// (optionally with gathered rows B[k][n] = B'[rb[k]][n]) or given by rows of
// R (B[k][n] = R[rb[n]][k], the transposed product of the
// reciprocity-symmetric operands used here).  A complex
// product is four real v_mfma_f64_16x16x4f64 products into separate real and
// imaginary accumulators.  Operand layouts of the 16x16x4 FP64 instruction:
// lane l holds A[l%16][l/16] and B[l/16][l%16]; accumulator register r holds
// D[l/16 + 4r][l%16] (measured: unlike the FP32 16x16x4 form, rows interleave).  Four waves per workgroup in a 2 x 2 arrangement, each
// owning WM x WN 16x16 blocks; K is staged through LDS 16 at a time.  A
// skinny product splits K over gridDim.z into a workspace reduced in a fixed
// order (deterministic).
//
// Block Woodbury (eq. lru_woodbury with M = |F|): after the pixels F flip,
// C_new = C_ref - U V^T with U = k0^2 G[:,F] diag(delta_F), V = I[:,F], so
//     C_new^-1 = C_ref^-1 + P Cap^-1 Q,   P = C_ref^-1 U,  Q = C_ref^-1[F,:],
//     Cap = I - Q U = I - P[F,:].
#include <algorithm>
#include <utility>

#include "dev_state.h"
#include "np_block.h"

namespace pngf {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGemmBK = 16;
constexpr size_t kNpSoloLds = 96 << 10;   // dynamic LDS that leaves room for one workgroup per CU


template <int WM, int WN, bool TRANSB, bool DINV = false>
__global__ __launch_bounds__(256) void k_zgemm(int M, int N, int K, const z64* A, int lda,
                                               const z64* B, int ldb, z64* C, int ldc,
                                               GemmIdx ix, z64 alpha, z64 beta, int kchunk,
                                               z64* work, NpDiag dg) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  __shared__ double sAr[BM][kGemmBK + 1], sAi[BM][kGemmBK + 1];
  __shared__ double sBr[kGemmBK][BN + 1], sBi[kGemmBK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int i16 = lane & 15, k4 = lane >> 4;
  // with a diagonal tile to invert, that tile's workgroup swaps places with
  // tile (0, 0), so it is dispatched first and its inverse starts earliest
  int bx = int(blockIdx.x), by = int(blockIdx.y);
  const bool diag = DINV && dg.tile >= 0;
  if (diag && bx == 0 && by == 0) {
    bx = dg.tile;
    by = dg.tile;
  } else if (diag && bx == dg.tile && by == dg.tile) {
    bx = 0;
    by = 0;
  }
  const int m0 = by * BM, n0 = bx * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  d4 accr[WM][WN], acci[WM][WN];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      accr[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      acci[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // the next K chunk is fetched into registers while the current one is
  // multiplied out of LDS.  The optional index maps are read first, then
  // every element's load is issued unconditionally (an element outside the
  // matrix loads a clamped in-range address and is replaced by zero), so that
  // no wait for one load sits between the others.
  constexpr int kAe = BM * kGemmBK / 256, kBe = BN * kGemmBK / 256;
  z64 ra[kAe], rbv[kBe];
  auto fetch = [&](int k0) {
    int ar_[kAe], ac_[kAe], br_[kBe], bc_[kBe];
    bool aok[kAe], bok[kBe];
#pragma unroll
    for (int q = 0; q < kAe; ++q) {
      const int e = tid + 256 * q;
      const int gr = m0 + (e >> 4), gc = k0 + (e & 15);
      aok[q] = gr < M && gc < kend;
      ar_[q] = min(gr, M - 1);
      ac_[q] = min(gc, K - 1);
    }
#pragma unroll
    for (int q = 0; q < kBe; ++q) {
      const int e = tid + 256 * q;
      // TRANSB: B is N x K (row n, column k); else K x N (row k, column n)
      const int gr = TRANSB ? n0 + (e >> 4) : k0 + e / BN;
      const int gc = TRANSB ? k0 + (e & 15) : n0 + e % BN;
      bok[q] = TRANSB ? (gr < N && gc < kend) : (gr < kend && gc < N);
      br_[q] = TRANSB ? min(gr, N - 1) : min(gr, K - 1);
      bc_[q] = TRANSB ? min(gc, K - 1) : min(gc, N - 1);
    }
    if (ix.ra) {
#pragma unroll
      for (int q = 0; q < kAe; ++q) ar_[q] = ix.ra[ar_[q]];
    }
    if (ix.ca) {
#pragma unroll
      for (int q = 0; q < kAe; ++q) ac_[q] = ix.ca[ac_[q]];
    }
    if (ix.rb) {
#pragma unroll
      for (int q = 0; q < kBe; ++q) br_[q] = ix.rb[br_[q]];
    }
    if (ix.cb) {
#pragma unroll
      for (int q = 0; q < kBe; ++q) bc_[q] = ix.cb[bc_[q]];
    }
#pragma unroll
    for (int q = 0; q < kAe; ++q) {
      const z64 v = A[size_t(ar_[q]) * lda + ac_[q]];
      ra[q] = aok[q] ? v : z64{0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < kBe; ++q) {
      const z64 v = B[size_t(br_[q]) * ldb + bc_[q]];
      rbv[q] = bok[q] ? v : z64{0.0, 0.0};
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kGemmBK) {
#pragma unroll
    for (int q = 0; q < kAe; ++q) {
      const int e = tid + 256 * q;
      sAr[e >> 4][e & 15] = ra[q].re;
      sAi[e >> 4][e & 15] = ra[q].im;
    }
#pragma unroll
    for (int q = 0; q < kBe; ++q) {
      const int e = tid + 256 * q;
      if (TRANSB) {
        sBr[e & 15][e >> 4] = rbv[q].re;
        sBi[e & 15][e >> 4] = rbv[q].im;
      } else {
        sBr[e / BN][e % BN] = rbv[q].re;
        sBi[e / BN][e % BN] = rbv[q].im;
      }
    }
    __syncthreads();
    if (k0 + kGemmBK < kend) fetch(k0 + kGemmBK);
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 4) {
      double ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int a = 0; a < WM; ++a) {
        const int r = wm * 16 * WM + a * 16 + i16;
        ar[a] = sAr[r][kk + k4];
        ai[a] = sAi[r][kk + k4];
      }
#pragma unroll
      for (int b = 0; b < WN; ++b) {
        const int n = wn * 16 * WN + b * 16 + i16;
        br[b] = sBr[kk + k4][n];
        bi[b] = sBi[kk + k4][n];
      }
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b) {
          accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], accr[a][b], 0, 0, 0);
          accr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], bi[b], accr[a][b], 0, 0, 0);
          acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acci[a][b], 0, 0, 0);
          acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acci[a][b], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const bool beta0 = beta.re == 0.0 && beta.im == 0.0;
  if (work) {
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int b = 0; b < WN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * 16 * WM + a * 16 + k4 + 4 * r;
          const int col = n0 + wn * 16 * WN + b * 16 + i16;
          if (row < M && col < N)
            work[(size_t(blockIdx.z) * M + row) * N + col] = z64{accr[a][b][r], acci[a][b][r]};
        }
  } else {
    // the lane's old C values are all requested before any is used (one
    // memory round trip, not one per element: a store to C could otherwise
    // alias the next load); the optional index maps are read first, and a
    // lane outside the matrix reads C[0] instead of branching around its load
    int crow[WM][4], ccol[WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 16 * WM + a * 16 + k4 + 4 * r;
        crow[a][r] = row < M ? (ix.rc ? ix.rc[row] : row) : -1;
      }
#pragma unroll
    for (int b = 0; b < WN; ++b) {
      const int col = n0 + wn * 16 * WN + b * 16 + i16;
      ccol[b] = col < N ? (ix.cc ? ix.cc[col] : col) : -1;
    }
    z64 old[WM][WN][4];
    if (!beta0) {
#pragma unroll
      for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool ok = crow[a][r] >= 0 && ccol[b] >= 0;
            old[a][b][r] = C[ok ? size_t(crow[a][r]) * ldc + ccol[b] : 0];
          }
    }
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
      for (int b = 0; b < WN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (crow[a][r] < 0 || ccol[b] < 0) continue;
          const z64 av = zmul(alpha, z64{accr[a][b][r], acci[a][b][r]});
          C[size_t(crow[a][r]) * ldc + ccol[b]] = beta0 ? av : zfma(beta, old[a][b][r], av);
        }
  }
  if (diag && bx == dg.tile && by == dg.tile) {
    // this workgroup's tile is the next diagonal block of the unpivoted
    // inversion: invert it now, from memory (the fence makes the tile's
    // stores visible to this workgroup's loads)
    __threadfence();
    __syncthreads();
    np_block_inverse<kNpNb>(C, ldc, dg.k0, dg.nb, dg.Bi, dg.status);
  }
}

// C = beta C + alpha sum_z work[z] (fixed summation order).
__global__ __launch_bounds__(256) void k_zgemm_reduce(int M, int N, int nz, const z64* work,
                                                      z64* C, int ldc, GemmIdx ix, z64 alpha,
                                                      z64 beta) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= size_t(M) * N) return;
  const int row = int(e / N), col = int(e % N);
  z64 s{0.0, 0.0};
  for (int z = 0; z < nz; ++z) s = zadd(s, work[size_t(z) * M * N + e]);
  z64* c = C + size_t(ix.rc ? ix.rc[row] : row) * ldc + (ix.cc ? ix.cc[col] : col);
  const z64 av = zmul(alpha, s);
  *c = (beta.re == 0.0 && beta.im == 0.0) ? av : zfma(beta, *c, av);
}

// P[:, c] *= s_c for the N_d x k panel P (s_c = k0^2 delta_c), then
// Cap[a][c] = delta_ac - P[F_a][c].
__global__ __launch_bounds__(256) void k_wood_scale(z64* P, int ldp, int nd, int k,
                                                    const double* s) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= size_t(nd) * k) return;
  const int i = int(e / k), c = int(e % k);
  P[size_t(i) * ldp + c] = zscale(P[size_t(i) * ldp + c], s[c]);
}
// kdev (nullable): the number of real flips on the device, the rest of the
// k entries being padding (pixel 0, scale 0): their rows of Cap are identity
// rows (their columns already are), and a count above k is reported as
// status 4.
__global__ __launch_bounds__(256) void k_wood_cap(const z64* P, int ldp, const int32_t* F, int k,
                                                  z64* Cap, int32_t* status,
                                                  const int32_t* kdev) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  // before the capacitance inverse reports
  if (status && e == 0) *status = (kdev && *kdev > k) ? 4 : 0;
  if (e >= k * k) return;
  const int a = e / k, c = e % k;
  if (kdev && a >= *kdev) {
    Cap[e] = z64{a == c ? 1.0 : 0.0, 0.0};
    return;
  }
  const z64 p = P[size_t(F[a]) * ldp + c];
  Cap[e] = z64{(a == c ? 1.0 : 0.0) - p.re, -p.im};
}

// Inverse of a k x k complex matrix (k <= kSmallInv), in place in A, by
// Gauss-Jordan elimination with partial pivoting.  One workgroup; the matrix
// ping-pongs between two LDS copies, so a column costs two barriers: wave 0
// picks the pivot row p, then every thread writes one entry of the next copy,
// with rows c and p exchanged on the way (M[c] <- M[p] / piv with 1 / piv in
// column c; M[r] <- M[r] - M[r][c] M[c] / piv with -M[r][c] / piv in column c).
// The column interchanges implied by the row exchanges are undone at the end
// in one pass.  status is set on a zero pivot.
constexpr int kSmallInv = 64;
constexpr int kSmallInvThreads = 256;

__global__ __launch_bounds__(kSmallInvThreads) void k_small_inverse(z64* A, int k, int32_t* status) {
  __shared__ z64 M[2][kSmallInv][kSmallInv + 1];
  __shared__ int perm[kSmallInv];
  __shared__ int cmap[kSmallInv];
  __shared__ int s_p;
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += kSmallInvThreads) M[0][e / k][e % k] = A[e];
  __syncthreads();
  int cur = 0;
  for (int c = 0; c < k; ++c) {
    const z64 (*X)[kSmallInv + 1] = M[cur];
    z64 (*Y)[kSmallInv + 1] = M[cur ^ 1];
    // pivot: largest |X[r][c]| over r >= c (the first of equals)
    if (tid < 64) {
      double best = -1.0;
      int bidx = k;
      for (int r = c + tid; r < k; r += 64) {
        const double a = zabs2(X[r][c]);
        if (a > best) { best = a; bidx = r; }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bidx, o, 64);
        if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
      }
      if (tid == 0) {
        if (!(best > 0.0)) {
          atomicOr(status, 1);
          bidx = c;
        }
        s_p = bidx;
        perm[c] = bidx;
      }
    }
    __syncthreads();
    const int p = s_p;
    const z64 piv = X[p][c];
    const z64 inv = zabs2(piv) > 0.0 ? zdiv(z64{1.0, 0.0}, piv) : z64{0.0, 0.0};
    for (int e = tid; e < k * k; e += kSmallInvThreads) {
      const int r = e / k, j = e % k;
      const z64 prow = (j == c) ? inv : zmul(X[p][j], inv);   // new pivot row
      if (r == c) {
        Y[c][j] = prow;
      } else {
        const int sr = (r == p) ? c : r;      // row r of the exchanged matrix
        const z64 f = X[sr][c];
        const z64 old = (j == c) ? z64{0.0, 0.0} : X[sr][j];
        Y[r][j] = zsub(old, zmul(f, prow));
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  // the row exchanges of columns c (rows c, perm[c]) become column exchanges
  // of the inverse, undone last first: cmap[j] = source column of column j
  if (tid == 0) {
    for (int j = 0; j < k; ++j) cmap[j] = j;
    for (int c = k - 1; c >= 0; --c) {
      const int q = perm[c];
      const int tmp = cmap[c];
      cmap[c] = cmap[q];
      cmap[q] = tmp;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += kSmallInvThreads) A[e] = M[cur][e / k][cmap[e % k]];
}

// The same inverse for k <= kWaveInv by four waves, with no row ever moved:
// column c takes as pivot p_c the row, not yet a pivot, with the largest
// |a_rc| (compared as the float of |a_rc|^2; the first of equals), and the
// in-place result M then satisfies A^-1[c][p_l] = M[p_c][l] (Gauss-Jordan on
// the row-permuted matrix, its rows left where they are).  Wave v holds
// columns [8v, 8v + 8), lane (r, h) = (lane % 32, lane / 32) the four
// entries [8v + 4h, 8v + 4h + 4) of row r in registers.  Column C is
// prepared by the wave that holds it, right after its own update for column
// C - 1: the pivot p (a DPP maximum of (|a|^2, row) keys), 1/a_pC (hardware
// reciprocal and two Newton steps) and every row's entry a_rC go to LDS (two
// copies by parity, so one barrier per column).  Every wave then takes the
// pivot row's entries of its own columns from lanes p and p + 32
// (cross-lane permute) and forms a <- alpha a + beta u for its four entries
// per lane, u the pivot row: alpha = 0 and beta = 1/p for the pivot row (the
// row scaled, 1/p in column C), alpha = 1 and beta = -a_iC/p elsewhere
// (column C becomes -a_iC/p, every other entry is reduced).  Columns run in
// groups of four (a loop), the four of a group unrolled so that a lane's
// entry in column C is a fixed register.  status is set on a zero pivot.
constexpr int kWaveInv = 32;

struct WgInvLds {
  z64 fac[2][kWaveInv];   // every row's entry in the pivot column
  z64 inv[2];             // 1 / pivot
  int p[2];               // pivot row
  int pv[kWaveInv];       // pivot row of each column
  int rowq[kWaveInv];     // column each row is the pivot of (-1: none)
};

// Posts column C's pivot row, 1 / pivot and the column's entries (run by
// the wave holding column C; x = the lane's entry in column C).
__device__ __forceinline__ void wg_inv_post(z64 x, int C, int k, int r, int h, int lane,
                                            uint32_t used, WgInvLds& sm) {
  const int b = C & 1;
  const int hs = (C >> 2) & 1;
  uint32_t key = 0;
  if (h == hs && r < k && !((used >> r) & 1u))
    key = (__float_as_uint(float(zabs2(x))) & ~31u) | uint32_t(31 - r);
  const int p = 31 - int(wave_max_u32(key) & 31u);
  const int pl = p + 32 * hs;
  const z64 apc{lane_d(x.re, pl), lane_d(x.im, pl)};
  if (h == hs) sm.fac[b][r] = x;
  if (lane == 0) {
    sm.p[b] = p;
    sm.inv[b] = zrecip_newton(apc);   // 0 for a zero pivot
  }
}

// Column C = 4 g + RC.
template <int RC>
__device__ __forceinline__ void wg_inv_step(z64 (&a)[4], int g, int k, int r, int h, int lane,
                                            int wv, int c0, uint32_t& used, WgInvLds& sm,
                                            int32_t* status) {
  const int C = 4 * g + RC;
  if (C >= k) return;
  lds_barrier();
  const int b = C & 1;
  const int p = sm.p[b];
  const z64 inv = sm.inv[b];
  const z64 f = sm.fac[b][r];
  if (threadIdx.x == 0) {
    if (!(zabs2(inv) > 0.0)) atomicOr(status, 1);   // zero pivot
    sm.pv[C] = p;
    sm.rowq[p] = C;
  }
  // the next column's entry first: the wave holding that column posts it
  // as soon as it is updated
  const int src = p + 32 * h;
  z64 u[4];
#pragma unroll
  for (int o = 1; o <= 4; ++o) u[(RC + o) & 3] = lane_bperm(a[(RC + o) & 3], src);
  used |= 1u << p;
  const bool piv = r == p;
  const bool mycol = c0 == 4 * g;   // this lane holds column C (as entry RC)
  const z64 fi = zmul(f, inv);
  const z64 beta = piv ? inv : z64{-fi.re, -fi.im};
#pragma unroll
  for (int o = 1; o <= 4; ++o) {
    const int q = (RC + o) & 3;
    const z64 x = piv ? z64{0.0, 0.0} : a[q];
    const z64 y = zfma(beta, u[q], x);
    // column C itself: 0 reduced by beta times the unit entry of the row
    a[q] = (q == RC && mycol) ? beta : y;
  }
  if (C + 1 < k && wv == ((C + 1) >> 3))
    wg_inv_post(a[(RC + 1) & 3], C + 1, k, r, h, lane, used, sm);
}

__global__ __launch_bounds__(256) void k_small_inverse_wg(z64* A, int k, int32_t* status) {
  __shared__ WgInvLds sm;
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  const int r = lane & 31, h = lane >> 5;
  const int c0 = 8 * wv + 4 * h;   // this lane's first column
  z64 a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    a[q] = (r < k && c0 + q < k) ? A[r * k + c0 + q] : z64{0.0, 0.0};
  if (t < kWaveInv) sm.rowq[t] = -1;
  uint32_t used = 0;   // rows already pivots (the same in every lane)
  if (wv == 0) wg_inv_post(a[0], 0, k, r, h, lane, used, sm);
#pragma unroll 1
  for (int g = 0; 4 * g < k; ++g) {
    wg_inv_step<0>(a, g, k, r, h, lane, wv, c0, used, sm, status);
    wg_inv_step<1>(a, g, k, r, h, lane, wv, c0, used, sm, status);
    wg_inv_step<2>(a, g, k, r, h, lane, wv, c0, used, sm, status);
    wg_inv_step<3>(a, g, k, r, h, lane, wv, c0, used, sm, status);
  }
  lds_barrier();
  if (r < k) {
    const int q = sm.rowq[r];
    if (q >= 0)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (c0 + e < k) A[q * k + sm.pv[c0 + e]] = a[e];
  }
}

// ------------------------------------------------------------------ launchers
// C = beta C + alpha A op(B) with the index maps of ix (see GemmIdx).
// work (>= splits * M * N entries) is used when splits > 1.
// nz_out (nullable): with more than one split, the partial products are
// left in work (work[z][row][col], z < *nz_out) for the caller to reduce.
hipError_t launch_zgemm_ix(int M, int N, int K, const z64* A, int lda, const z64* B, int ldb,
                           bool transb, z64* C, int ldc, const GemmIdx& ix, z64 alpha, z64 beta,
                           int splits, z64* work, hipStream_t s, int* nz_out) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K <= 0) return hipErrorInvalidValue;
  splits = std::max(1, std::min(splits, (K + kGemmBK - 1) / kGemmBK));
  if (splits > 1 && !work) return hipErrorInvalidValue;
  int kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kGemmBK - 1) / kGemmBK * kGemmBK;
  splits = (K + kchunk - 1) / kchunk;
  z64* wk = splits > 1 ? work : nullptr;
  // 64 x 64 tiles for large products; a rank-k update (short K) is bound by
  // reading and writing C, and its 32 x 32 tiles (fewer registers, four
  // times the workgroups) keep more of them in flight
  const bool big = M >= 512 && N >= 512 && K > 64;
  if (big) {
    dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
    if (transb)
      hipLaunchKernelGGL((k_zgemm<2, 2, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                         ldc, ix, alpha, beta, kchunk, wk, NpDiag{});
    else
      hipLaunchKernelGGL((k_zgemm<2, 2, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                         ldc, ix, alpha, beta, kchunk, wk, NpDiag{});
  } else {
    dim3 grid((N + 31) / 32, (M + 31) / 32, splits);
    if (transb)
      hipLaunchKernelGGL((k_zgemm<1, 1, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                         ldc, ix, alpha, beta, kchunk, wk, NpDiag{});
    else
      hipLaunchKernelGGL((k_zgemm<1, 1, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                         ldc, ix, alpha, beta, kchunk, wk, NpDiag{});
  }
  if (nz_out) *nz_out = splits > 1 ? splits : 0;
  if (splits > 1 && !nz_out) {
    const size_t n = size_t(M) * N;
    hipLaunchKernelGGL(k_zgemm_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, M, N,
                       splits, work, C, ldc, ix, alpha, beta);
  }
  return hipGetLastError();
}

// The rank-nb update of the unpivoted inversion, C += A B (64 x 64 tiles,
// which line up with its panels), with the diagonal tile dg inverted by its
// own workgroup.
hipError_t launch_zgemm_np(int M, int N, int K, const z64* A, int lda, const z64* B, int ldb,
                           z64* C, int ldc, const NpDiag& dg, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  static_assert(kNpNb == 64, "panel width equals the GEMM tile");
  dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
  // a small update, whose tiles the chip runs in a round or two, reserves
  // enough LDS for one workgroup per CU, so that no other tile shares the
  // CU of the diagonal tile's inverse (on the critical path); a large one
  // keeps its occupancy
  const size_t lds = (dg.tile >= 0 && size_t(grid.x) * grid.y <= 512) ? kNpSoloLds : 0;
  hipLaunchKernelGGL((k_zgemm<2, 2, false, true>), grid, dim3(256), lds, s, M, N, K, A, lda, B,
                     ldb, C, ldc, GemmIdx{}, z64{1.0, 0.0}, z64{1.0, 0.0}, K, nullptr, dg);
  return hipGetLastError();
}

// Common case: column gather of A (ca) and row gather of B (rb: rows of R
// by n when transb, rows of B by k otherwise).
hipError_t launch_zgemm(int M, int N, int K, const z64* A, int lda, const int32_t* ca,
                        const z64* B, int ldb, bool transb, const int32_t* rb, z64* C, int ldc,
                        z64 alpha, z64 beta, int splits, z64* work, hipStream_t s, int* nz_out) {
  GemmIdx ix;
  ix.ca = ca;
  ix.rb = rb;
  return launch_zgemm_ix(M, N, K, A, lda, B, ldb, transb, C, ldc, ix, alpha, beta, splits, work, s,
                         nz_out);
}

// The block-Woodbury panel from the skinny GEMM's partial products, in one
// pass: P[i][c] = s_c sum_z work[z][i][c] (fixed order), and the capacitance
// matrix Cap[a][c] = delta_ac - P[F_a][c] from the same sums; status
// (nullable) is cleared first.  Same arithmetic as k_zgemm_reduce followed
// by k_wood_scale and k_wood_cap.
__global__ __launch_bounds__(256) void k_wood_panel(const z64* work, int nz, int nd, int k,
                                                    const double* sc, z64* P, int ldp,
                                                    const int32_t* F, z64* Cap,
                                                    int32_t* status, const int32_t* kdev) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  const size_t np = size_t(nd) * k;
  if (status && e == 0) *status = (kdev && *kdev > k) ? 4 : 0;
  if (e < np) {
    z64 v{0.0, 0.0};
    for (int z = 0; z < nz; ++z) v = zadd(v, work[size_t(z) * np + e]);
    const int i = int(e / k), c = int(e % k);
    P[size_t(i) * ldp + c] = zscale(zmul(z64{1.0, 0.0}, v), sc[c]);
  } else if (e < np + size_t(k) * k) {
    const int q = int(e - np), a = q / k, c = q % k;
    if (kdev && a >= *kdev) {   // a padding row (see k_wood_cap)
      Cap[q] = z64{a == c ? 1.0 : 0.0, 0.0};
      return;
    }
    const size_t src = size_t(F[a]) * k + c;
    z64 v{0.0, 0.0};
    for (int z = 0; z < nz; ++z) v = zadd(v, work[size_t(z) * np + src]);
    const z64 p = zscale(zmul(z64{1.0, 0.0}, v), sc[c]);
    Cap[q] = z64{(a == c ? 1.0 : 0.0) - p.re, -p.im};
  }
}

hipError_t launch_wood_panel(const z64* work, int nz, int nd, int k, const double* sc, z64* P,
                             int ldp, const int32_t* F, z64* Cap, int32_t* status, hipStream_t s,
                             const int32_t* kdev) {
  if (k <= 0) return hipSuccess;
  const size_t n = size_t(nd) * k + size_t(k) * k;
  hipLaunchKernelGGL(k_wood_panel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, work, nz, nd,
                     k, sc, P, ldp, F, Cap, status, kdev);
  return hipGetLastError();
}

// status (nullable) is cleared before the capacitance matrix is formed.
hipError_t launch_wood_cap(z64* P, int ldp, int nd, const int32_t* F, int k, const double* sc,
                           z64* Cap, int32_t* status, hipStream_t s, const int32_t* kdev) {
  if (k <= 0) return hipSuccess;
  const size_t n = size_t(nd) * k;
  hipLaunchKernelGGL(k_wood_scale, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, P, ldp, nd, k,
                     sc);
  hipLaunchKernelGGL(k_wood_cap, dim3((k * k + 255) / 256), dim3(256), 0, s, P, ldp, F, k, Cap,
                     status, kdev);
  return hipGetLastError();
}

hipError_t launch_small_inverse(z64* A, int k, int32_t* status, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (k > kSmallInv) return hipErrorInvalidValue;
  if (k <= kWaveInv)
    hipLaunchKernelGGL(k_small_inverse_wg, dim3(1), dim3(256), 0, s, A, k, status);
  else
    hipLaunchKernelGGL(k_small_inverse, dim3(1), dim3(kSmallInvThreads), 0, s, A, k, status);
  return hipGetLastError();
}

}  // namespace pngf
