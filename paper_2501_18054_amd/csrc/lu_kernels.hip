// FP64 direct inversion of the PNGF system matrix on the GPU (gfx950).
//
// Used for the initial inverse C0^-1 (Direct binary search: the inverse of the
// initial system matrix is found and stored) and for the periodic
// re-inversion that bounds the drift of long chains of low-rank updates
// (Computational efficiency: direct re-inversion instead of Woodbury when many
// unknowns have changed).
//
// Structure.  C = I - k0^2 G diag(deps) has an identity column for every pixel
// with deps = 0.  With S the pixels at eps_hi and Z the others,
//     C = [[K, 0], [W, I]],  K = I - k0^2 deps G[S,S],  W = -k0^2 deps G[Z,S],
//     C^-1 = [[K^-1, 0], [k0^2 deps G[Z,S] K^-1, I]],
// so only K (|S| ~ N_d/2) is inverted, and the Z rows are one GEMM.  This is
// the field-form counterpart of the paper's system (I - P) + P G, whose rows
// for empty tiles are identity rows (Results, Numerical Green's functions).
//
// K^-1 by blocked Gauss-Jordan elimination with partial pivoting, in place.
// Pivoting is virtual (rows never move): column k uses pivot row p_k, so the
// elimination is that of Pi K with (Pi K)[k,:] = K[p_k,:], the in-place result
// M satisfies (Pi K)^-1[k,:] = M[p_k,:], and K^-1[i, p_l] = M[p_i, l].
// A panel of kGjNb columns picks its pivot rows by partial pivoting over
// every candidate row in one workgroup (rows in registers, one LDS exchange
// per column).  Above kGeppRows rows the candidates are first thinned by
// tournament pivoting (Grigori-Demmel-Xiang CALU): groups of 64 rows, one
// group per wave across the chip, each propose kGjNb rows by the same
// elimination; the proposals of four groups form the next level's group
// until one workgroup can take them all.  The winners' block B11 is inverted
// and every row is reduced independently, giving the Gauss-Jordan panel
// [-B01 B11^-1; B11^-1; -B21 B11^-1].  Every column outside the panel then gets the rank-kGjNb
// update M[r,j] = (r pivot of this panel ? 0 : M[r,j]) + P[r,:] B1[:,j] with
// B1 the panel's pivot rows before the update (the reduction of the panel
// rows happens inside the update's workgroups, and the new pivot rows wait
// in a side buffer until the next panel's update, so no workgroup reads a
// row another one writes).  On gfx950 the FP64
// matrix-core rate equals the FP64 vector rate (78.6 TFLOP/s), and at this
// panel width the update is HBM-bound, so it runs on the vector ALUs.
#include <utility>

#include "dev_state.h"
#include "np_block.h"

namespace pngf {

hipError_t launch_zgemm_ix(int M, int N, int K, const z64* A, int lda, const z64* B, int ldb,
                           bool transb, z64* C, int ldc, const GemmIdx& ix, z64 alpha, z64 beta,
                           int splits, z64* work, hipStream_t s, int* nz_out = nullptr);
hipError_t launch_zgemm_np(int M, int N, int K, const z64* A, int lda, const z64* B, int ldb,
                           z64* C, int ldc, const NpDiag& dg, hipStream_t s);

constexpr int kGjNb = 16;
constexpr int kUpdRows = 16;      // rows per update workgroup (small systems)
constexpr int kUpdRowsBig = 64;   // ... from kUpdBigFrom pivot rows on: the pivot rows'
constexpr int kUpdBigFrom = 2048; // values and the panel factors are shared by more rows
constexpr int kGeppRows = 1024;   // candidates one partial-pivoting workgroup takes
constexpr int kNpFoldMax = 2048;  // largest n_S whose Z rows ride along in the panel updates

// K[a][b] = delta_ab - k2d G[s_a][s_b]; clears the pivot marks.
__global__ __launch_bounds__(256) void k_gather_K(z64* K, const z64* G, int ld, const int32_t* sidx,
                                                  int ns, double k2d, int32_t* used) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= ns) return;
  const z64 g = G[size_t(sidx[a]) * ld + sidx[b]];
  K[size_t(a) * ld + b] = z64{(a == b ? 1.0 : 0.0) - k2d * g.re, -k2d * g.im};
  if (a == 0) used[b] = 0;
}

// Panel columns [k0, k0+ncols) gathered into a contiguous buffer, column
// by column (entry (r, c) at Pb[c n + r]), so that consecutive rows of one
// column are adjacent for the pivot search's loads.
__global__ __launch_bounds__(256) void k_gj_panel_in(const z64* S, int ld, int n, int k0,
                                                     int ncols, z64* Pb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int c = e / n, r = e % n;
  if (c < kGjNb) Pb[e] = (c < ncols) ? S[size_t(r) * ld + k0 + c] : z64{0.0, 0.0};
}

// Broadcast of lane p's value to the wave (p wave-uniform).
__device__ __forceinline__ float lane_f(float v, int p) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), p));
}

// Elimination column C of a one-wave tournament group (rows in registers,
// one per lane): the live row of largest |a_C|^2 pivots (the lowest lane on
// ties; key 0 marks a lane with no live row), its row is broadcast by
// readlane and every row is reduced by it.  Rows that are no longer live are
// reduced too: nothing reads them again.
template <int C>
__device__ __forceinline__ void wt_column(z32 (&a)[kGjNb], bool& alive, int lane, int nsel,
                                          int& order, bool& zero) {
  if (C >= nsel) return;
  const float m = a[C].re * a[C].re + a[C].im * a[C].im;
  const uint32_t key = alive ? __float_as_uint(m) + 1u : 0u;
  const uint32_t mx = wave_max_u32(key);
  const unsigned long long hit = __ballot(key == mx);
  const int p = __builtin_amdgcn_readfirstlane(__ffsll(static_cast<long long>(hit)) - 1);
  if (mx <= 1u) zero = true;
  if (lane == p) {
    order = C;
    alive = false;
  }
  const float pr = lane_f(a[C].re, p), pi = lane_f(a[C].im, p);
  const float d = pr * pr + pi * pi;
  const float sc = d > 0.f ? __builtin_amdgcn_rcpf(d) : 0.f;   // selection only: 1 ulp is enough
  const float ir = pr * sc, ii = -pi * sc;
  const float lr = a[C].re * ir - a[C].im * ii, li = a[C].re * ii + a[C].im * ir;
#pragma unroll
  for (int cc = C + 1; cc < kGjNb; ++cc) {
    const float ur = lane_f(a[cc].re, p), ui = lane_f(a[cc].im, p);
    a[cc].re = fmaf(li, ui, fmaf(-lr, ur, a[cc].re));
    a[cc].im = fmaf(-li, ur, fmaf(-lr, ui, a[cc].im));
  }
}

template <int... Cs>
__device__ __forceinline__ void wt_columns(z32 (&a)[kGjNb], bool& alive, int lane, int nsel,
                                           int& order, bool& zero,
                                           std::integer_sequence<int, Cs...>) {
  (wt_column<Cs>(a, alive, lane, nsel, order, zero), ...);
}

// One tournament group in one wave: candidate `row` of this lane (< 0: none)
// proposes min(ncols, #candidates) pivot rows by partial pivoting on
// complex-FP32 copies of the panel rows; writes them in pivot order to
// out[0..count) and the count to *cnt.  Returns whether a chosen pivot had
// magnitude zero.
__device__ __forceinline__ bool wave_tournament(const z64* Pb, int n, int ncols, int row,
                                                int lane, int* out, int* cnt) {
  z32 a[kGjNb];
#pragma unroll
  for (int c = 0; c < kGjNb; ++c) {
    z32 v{0.f, 0.f};
    if (row >= 0 && c < ncols) {
      const z64 x = Pb[size_t(c) * n + row];
      v = z32{float(x.re), float(x.im)};
    }
    a[c] = v;
  }
  bool alive = row >= 0;
  const int nsel = min(ncols, int(__popcll(__ballot(alive))));
  int order = -1;
  bool zero = false;
  wt_columns(a, alive, lane, nsel, order, zero, std::make_integer_sequence<int, kGjNb>{});
  if (order >= 0) out[order] = row;
  if (lane == 0) *cnt = nsel;
  return zero;
}

// One level of a panel's tournament spread over the chip, one group per
// one-wave workgroup g, proposals into cand[16g ..] and cnt[g].  Level 0
// (gin null): the rows [64g, 64g + 64) that are not yet pivots; a merge
// level: the proposals of groups 4g .. 4g+3 of the ngin in (gin, gcnt).
__global__ __launch_bounds__(64) void k_tsel_wave(const z64* Pb, int n, int ncols,
                                                  const int32_t* used, const int32_t* gin,
                                                  const int32_t* gcnt, int ngin, int32_t* cand,
                                                  int32_t* cnt) {
  const int lane = threadIdx.x, g = blockIdx.x;
  int row = -1;
  if (gin == nullptr) {
    row = g * 64 + lane;
    if (row >= n || used[row]) row = -1;
  } else {
    const int grp = g * 4 + lane / kGjNb, u = lane % kGjNb;
    if (grp < ngin && u < gcnt[grp]) row = gin[grp * kGjNb + u];
  }
  wave_tournament(Pb, n, ncols, row, lane, cand + g * kGjNb, cnt + g);
}

// Lane (16 g + q)'s value to every lane of its 16-lane row g (DPP
// row_newbcast), for a z64 held one per lane.
template <int Q>
__device__ __forceinline__ z64 row_bcast(z64 v) {
  const unsigned long long r = static_cast<unsigned long long>(__double_as_longlong(v.re));
  const unsigned long long i = static_cast<unsigned long long>(__double_as_longlong(v.im));
  auto b = [](uint32_t x) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x150 | Q, 0xF, 0xF, false));
  };
  const uint64_t r2 = (uint64_t(b(uint32_t(r >> 32))) << 32) | b(uint32_t(r));
  const uint64_t i2 = (uint64_t(b(uint32_t(i >> 32))) << 32) | b(uint32_t(i));
  return z64{__longlong_as_double(static_cast<long long>(r2)),
             __longlong_as_double(static_cast<long long>(i2))};
}

// LDS of the one-workgroup pivot search.  The keys cycle through three
// buffers (column C uses C % 3): a key is cleared by thread 0 right after
// the barrier that follows its last reads, two barriers before its next
// use.  Every wave's candidate row of every column is kept (val), so the
// winners' rows are the in-place LU of B11 without a copy.
struct GeppLds {
  unsigned long long key[3];
  int win[kGjNb];
  int wsel[kGjNb];
  z64 val[kGjNb][16][kGjNb];
};

// Column C of the one-workgroup partial pivoting below, in FP64 on in-place
// LU rows (entries left of C hold the row's multipliers, the rest its
// reduced values).  Each wave reduces its key (the high word of |a_C|^2 + 1
// for a live row, 0 for none: a 20-bit mantissa suffices to pick a pivot)
// by DPP, and its best lane posts the key with the wave id and the row id
// below it by one LDS 64-bit max (largest magnitude, then lowest wave wins)
// and its row by plain stores; after the barrier one LDS read names the
// winner, whose row every thread reads by broadcast to form its multiplier
// (kept in a[C]) and reduce the rest of its row.
template <int C>
__device__ __forceinline__ void gepp_column(z64 (&a)[kGjNb], int row, bool& alive, int lane,
                                            int wid, int nsel, GeppLds& sh, bool& zero) {
  if (C >= nsel) return;
  constexpr int buf = C % 3;
  const double m = a[C].re * a[C].re + a[C].im * a[C].im;
  const uint32_t key = alive ? uint32_t(__double_as_longlong(m) >> 32) + 1u : 0u;
  const uint32_t mx = wave_max_u32(key);
  const int p = __builtin_amdgcn_readfirstlane(
      __ffsll(static_cast<long long>(__ballot(key == mx))) - 1);
  if (lane == p && mx != 0u) {
    atomicMax(&sh.key[buf], (static_cast<unsigned long long>(mx) << 32) |
                                (uint32_t(15 - wid) << 24) | uint32_t(row));
#pragma unroll
    for (int q = 0; q < kGjNb; ++q) sh.val[C][wid][q] = a[q];
  }
  lds_barrier();
  const unsigned long long k64 = sh.key[buf];
  const uint32_t gm = uint32_t(k64 >> 32);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(k64));
  const int w = 15 - int(lo >> 24);
  const int prow = int(lo & 0xFFFFFFu);
  if (gm <= 1u) zero = true;
  if (wid == 0 && lane == 0) {
    sh.win[C] = prow;
    sh.wsel[C] = w;
    sh.key[(C + 2) % 3] = 0ull;
  }
  const z64 l = zmul(a[C], zrecip_newton(sh.val[C][w][C]));
  if (row == prow) alive = false;
  a[C] = l;
#pragma unroll
  for (int cc = C + 1; cc < kGjNb; ++cc) {
    const z64 u = sh.val[C][w][cc];
    a[cc].re = fma(-l.re, u.re, fma(l.im, u.im, a[cc].re));
    a[cc].im = fma(-l.re, u.im, fma(-l.im, u.re, a[cc].im));
  }
}

template <int... Cs>
__device__ __forceinline__ void gepp_columns(z64 (&a)[kGjNb], int row, bool& alive, int lane,
                                             int wid, int nsel, GeppLds& sh, bool& zero,
                                             std::integer_sequence<int, Cs...>) {
  (gepp_column<Cs>(a, row, alive, lane, wid, nsel, sh, zero), ...);
}

// Step Q of the two triangular solves of the finish (one column per 16-lane
// row, lane i of the row holding entry i): forward, x_i -= L[i][Q] x_Q for
// i > Q (L unit lower); backward, y_Q = x_Q / U[Q][Q], then x_i -= U[i][Q]
// y_Q for i < Q.
template <int Q>
__device__ __forceinline__ void fwd_step(z64& x, const z64 (&lu)[kGjNb], int i) {
  const z64 xq = row_bcast<Q>(x);
  if (i > Q) x = zsub(x, zmul(lu[Q], xq));
}
template <int Q>
__device__ __forceinline__ void bwd_step(z64& x, const z64 (&lu)[kGjNb], z64 invd, int i) {
  if (i == Q) x = zmul(x, invd);
  const z64 yq = row_bcast<Q>(x);
  if (i < Q) x = zsub(x, zmul(lu[Q], yq));
}
template <int... Qs>
__device__ __forceinline__ void fwd_steps(z64& x, const z64 (&lu)[kGjNb], int i,
                                          std::integer_sequence<int, Qs...>) {
  (fwd_step<Qs>(x, lu, i), ...);
}
template <int... Qs>
__device__ __forceinline__ void bwd_steps(z64& x, const z64 (&lu)[kGjNb], z64 invd, int i,
                                          std::integer_sequence<int, Qs...>) {
  (bwd_step<kGjNb - 1 - Qs>(x, lu, invd, i), ...);
}

// After the pivot search: B11^-1 = U^-1 L^-1 from the winners' LU rows
// (identity rows and columns pad a ragged panel), four columns per wave,
// column j in the 16-lane row j % 4 of wave j / 4 (waves take further
// columns if there are fewer than four).  Lane i of a row keeps row i of L
// and U in registers and solves L x = e_j, then U y = x, by broadcasts
// within the row.  Thread 0 writes piv and used.
__device__ __forceinline__ void gepp_finish(GeppLds& sh, int k0, int ncols, int nsel, int t,
                                            int nthreads, int32_t* piv, int32_t* used,
                                            z64* B11inv) {
  const int lane = t & 63, i = lane & 15;
  z64 lu[kGjNb];
#pragma unroll
  for (int q = 0; q < kGjNb; ++q) {
    z64 v{i == q ? 1.0 : 0.0, 0.0};
    if (i < nsel && q < nsel) v = sh.val[i][sh.wsel[i]][q];
    lu[q] = v;
  }
  const z64 invd = zrecip_newton(i < nsel ? sh.val[i][sh.wsel[i]][i] : z64{1.0, 0.0});
  for (int j = t >> 4; j < kGjNb; j += nthreads >> 4) {
    z64 x{i == j ? 1.0 : 0.0, 0.0};
    fwd_steps(x, lu, i, std::make_integer_sequence<int, kGjNb>{});
    bwd_steps(x, lu, invd, i, std::make_integer_sequence<int, kGjNb>{});
    B11inv[i * kGjNb + j] = x;
  }
  if (t < nsel) {
    const int rw = sh.win[t];
    piv[k0 + t] = rw;
    used[rw] = k0 + t + 1;
  }
}

// Partial pivoting of one panel in FP64 over every candidate row at once, in
// one workgroup of up to 16 waves: thread t holds candidate t's panel row in
// registers (the rows [0, n) that are not pivots yet if gin is null, else
// the proposals (gin, gcnt) of ngin tournament groups); every live row is
// reduced by each chosen pivot.  Then B11^-1, piv and used; a zero pivot is
// flagged in *status.
__global__ __launch_bounds__(1024) void k_tsel_gepp(const z64* Pb, int n, int k0, int ncols,
                                                    const int32_t* gin, const int32_t* gcnt,
                                                    int ngin, int32_t* piv, int32_t* used,
                                                    z64* B11inv, int32_t* status) {
  __shared__ GeppLds sh;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  if (t < 2) sh.key[t] = 0ull;
  int r = -1;
  if (gin == nullptr) {
    if (t < n && !used[t]) r = t;
  } else {
    const int grp = t / kGjNb, u = t % kGjNb;
    if (grp < ngin && u < gcnt[grp]) r = gin[grp * kGjNb + u];
  }
  z64 a[kGjNb];
#pragma unroll
  for (int q = 0; q < kGjNb; ++q)
    a[q] = (r >= 0 && q < ncols) ? Pb[size_t(q) * n + r] : z64{0.0, 0.0};
  bool alive = r >= 0;
  const int nsel = min(ncols, __syncthreads_count(alive));
  bool zero = false;
  gepp_columns(a, r, alive, lane, wid, nsel, sh, zero, std::make_integer_sequence<int, kGjNb>{});
  if (zero && t == 0) atomicOr(status, 1);
  __syncthreads();
  gepp_finish(sh, k0, ncols, nsel, t, int(blockDim.x), piv, used, B11inv);
}

// One partial-pivoting workgroup over m <= kGeppRows candidates.
void launch_tsel_gepp(const z64* Pb, int n, int k0, int ncols, const int32_t* gin,
                      const int32_t* gcnt, int ngin, int m, int32_t* piv, int32_t* used,
                      z64* B11inv, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_tsel_gepp, dim3(1), dim3(64 * ((m + 63) / 64)), 0, s, Pb, n, k0, ncols,
                     gin, gcnt, ngin, piv, used, B11inv, status);
}

// Rank-ncols update of one panel, with the panel's reduction by B11^-1
// folded in: each workgroup forms the reduced panel entries Pt of its rows
// from the gathered panel Pb (pivot rows, used[r]-1 in the panel: their row
// of B11^-1; every other row r: -B_r B11^-1).  Every workgroup reads the
// panel's pivot rows of S as they were before the update (b), so their new
// values go to PRc instead of S; the previous panel's pivot rows, held in
// PRp, are read from there and written back to S.  Panel columns get Pt; the
// next panel's columns (updated here) are also gathered into Pn.  A
// workgroup covers 64 columns x ROWS rows; thread (g, c) owns column c
// and rows g, g+4, ...
template <int ROWS>
__global__ __launch_bounds__(256) void k_gj_update(z64* S, int ld, int n, int k0, int ncols,
                                                   const int32_t* used, const int32_t* piv,
                                                   const z64* B11inv, const z64* Pb,
                                                   const z64* PRp, z64* PRc, z64* Pn) {
  static_assert(kGjNb * kGjNb == 256, "one B11^-1 entry per thread");
  __shared__ z64 Bi[kGjNb][kGjNb];
  __shared__ z64 R[ROWS][kGjNb + 1];
  __shared__ z64 Pt[ROWS][kGjNb + 1];
  // 1 + c: pivot c of this panel; -(1 + c): pivot c of the previous one; 0
  __shared__ int kind[ROWS];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.y * ROWS;
  Bi[tid / kGjNb][tid % kGjNb] = B11inv[tid];
  for (int e = tid; e < ROWS * kGjNb; e += 256) {
    const int c = e / ROWS, rr = e % ROWS;
    const int r = r0 + rr;
    R[rr][c] = (r < n && c < ncols) ? Pb[size_t(c) * n + r] : z64{0.0, 0.0};
  }
  if (tid < ROWS) {
    const int r = r0 + tid;
    const int u = (r < n) ? used[r] - 1 : -1;
    int kd = 0;
    if (u >= k0 && u < k0 + ncols) kd = 1 + (u - k0);
    else if (u >= 0 && u >= k0 - kGjNb && u < k0) kd = -(1 + u - (k0 - kGjNb));
    kind[tid] = kd;
  }
  __syncthreads();
  for (int e = tid; e < ROWS * kGjNb; e += 256) {
    const int rr = e / kGjNb, cc = e % kGjNb;
    z64 out{0.0, 0.0};
    if (cc < ncols) {
      if (kind[rr] > 0) {
        out = Bi[kind[rr] - 1][cc];
      } else {
        z64 acc{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < kGjNb; ++q) acc = zfma(R[rr][q], Bi[q][cc], acc);
        out = z64{-acc.re, -acc.im};
      }
    }
    Pt[rr][cc] = out;
  }
  __syncthreads();
  const int j = blockIdx.x * 64 + (tid & 63);
  const int rg = tid >> 6;
  if (j >= n) return;
  if (j >= k0 && j < k0 + ncols) {
    for (int rr = rg; rr < ROWS && r0 + rr < n; rr += 4) {
      const int kd = kind[rr];
      z64* dst = (kd > 0) ? PRc + size_t(kd - 1) * ld + j : S + size_t(r0 + rr) * ld + j;
      *dst = Pt[rr][j - k0];
    }
    return;
  }
  const int nxt = k0 + kGjNb;
  const bool in_next = (j >= nxt && j < nxt + kGjNb);
  z64 b[kGjNb];
#pragma unroll
  for (int c = 0; c < kGjNb; ++c)
    b[c] = (c < ncols) ? S[size_t(piv[k0 + c]) * ld + j] : z64{0.0, 0.0};
  for (int rr = rg; rr < ROWS && r0 + rr < n; rr += 4) {
    const int kd = kind[rr];
    z64* row = S + size_t(r0 + rr) * ld + j;
    z64 acc{0.0, 0.0};
    if (kd < 0) acc = PRp[size_t(-kd - 1) * ld + j];
    else if (kd == 0) acc = *row;
#pragma unroll
    for (int c = 0; c < kGjNb; ++c) acc = zfma(Pt[rr][c], b[c], acc);
    if (kd > 0) PRc[size_t(kd - 1) * ld + j] = acc;
    else *row = acc;
    if (in_next) Pn[size_t(j - nxt) * n + r0 + rr] = acc;
  }
}

// The last panel's pivot rows back from PR into S.
__global__ __launch_bounds__(256) void k_gj_rows_back(z64* S, int ld, int n, int k0, int ncols,
                                                      const int32_t* piv, const z64* PR) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (j < n && c < ncols) S[size_t(piv[k0 + c]) * ld + j] = PR[size_t(c) * ld + j];
}

// inv_p[p_l] = l
__global__ __launch_bounds__(256) void k_gj_invperm(const int32_t* piv, int32_t* inv_p, int n) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l < n) inv_p[piv[l]] = l;
}

// C^-1 rows of S: C^-1[s_a, j] = K^-1[a, pos[j]] = M[p_a][inv_p[pos[j]]] for
// j in S, 0 otherwise.  Rows of Z: identity on Z columns (the S columns come
// from the Z-rows GEMM).  One row per blockIdx.y.
__global__ __launch_bounds__(256) void k_scatter_inverse(const z64* M, z64* Cinv, int ld, int nd,
                                                         const int32_t* pos, const int32_t* piv,
                                                         const int32_t* inv_p) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nd) return;
  const int a = pos[i], bj = pos[j];
  z64 v{0.0, 0.0};
  if (a >= 0) {
    if (bj >= 0) v = M[size_t(piv[a]) * ld + inv_p[bj]];
    Cinv[size_t(i) * ld + j] = v;
  } else if (bj < 0) {
    Cinv[size_t(i) * ld + j] = z64{i == j ? 1.0 : 0.0, 0.0};
  }
}

// y[i] = beta w[i] + gamma w2[i] + alpha sum_j A[i,j] d_j v[j], with
// d_j = (bits[j] ? ds : 0) when bits != nullptr, else 1.  One workgroup per
// row; y may alias w (row i reads w[i] before writing y[i]).
// A32 (nullable): also writes the complex-FP32 copy of the row it reads.
// Each thread takes j = tid, tid + 256, ... in order, kGemvUnroll at a time:
// their loads are issued together (clamped in-range addresses, results past
// the row end unused), so a row costs a few memory round trips.
constexpr int kGemvUnroll = 4;

__global__ __launch_bounds__(kRowThreads) void k_gemv(const z64* A, int ld, int n, const z64* v,
                                                      const uint8_t* bits, double ds, z64 alpha,
                                                      z64 beta, const z64* w, double gamma,
                                                      const z64* w2, z64* y, z32* A32) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int i = blockIdx.x;
  const z64* a = A + size_t(i) * ld;
  z64 acc{0.0, 0.0};
  for (int j0 = threadIdx.x; j0 < n; j0 += kGemvUnroll * kRowThreads) {
    z64 aj[kGemvUnroll], vj[kGemvUnroll];
    uint32_t bj[kGemvUnroll];
    if (bits) {
#pragma unroll
      for (int u = 0; u < kGemvUnroll; ++u) bj[u] = bits[min(j0 + u * kRowThreads, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int j = min(j0 + u * kRowThreads, n - 1);
      aj[u] = a[j];
      vj[u] = v[j];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int j = j0 + u * kRowThreads;
      if (j < n) {
        if (A32) A32[size_t(i) * ld + j] = z32{float(aj[u].re), float(aj[u].im)};
        acc = zfma(aj[u], bits ? zscale(vj[u], bj[u] ? ds : 0.0) : vj[u], acc);
      }
    }
  }
  const z64 s = block_zsum(acc, red);
  if (threadIdx.x == 0) {
    z64 out = zmul(alpha, s);
    if (w) out = zfma(beta, w[i], out);
    if (w2) out = zadd(out, zscale(w2[i], gamma));
    y[i] = out;
  }
}

// Two products with one pass over A: for o in {o1, o2},
// o.y[i] = o.beta o.w[i] + o.gamma o.w2[i] + o.alpha sum_j A[i,j] d_j o.v[j]
// (d as in k_gemv).  o.y may alias o.w.
__global__ __launch_bounds__(kRowThreads) void k_gemv2(const z64* A, int ld, int n,
                                                       const uint8_t* bits, double ds, GemvOut o1,
                                                       GemvOut o2) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int i = blockIdx.x;
  const z64* a = A + size_t(i) * ld;
  z64 acc1{0.0, 0.0}, acc2{0.0, 0.0};
  for (int j0 = threadIdx.x; j0 < n; j0 += kGemvUnroll * kRowThreads) {
    z64 aj[kGemvUnroll], v1[kGemvUnroll], v2[kGemvUnroll];
    uint32_t bj[kGemvUnroll];
    if (bits) {
#pragma unroll
      for (int u = 0; u < kGemvUnroll; ++u) bj[u] = bits[min(j0 + u * kRowThreads, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int j = min(j0 + u * kRowThreads, n - 1);
      aj[u] = a[j];
      v1[u] = o1.v[j];
      v2[u] = o2.v[j];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      if (j0 + u * kRowThreads < n) {
        const double dj = bits ? (bj[u] ? ds : 0.0) : 1.0;
        acc1 = zfma(aj[u], zscale(v1[u], dj), acc1);
        acc2 = zfma(aj[u], zscale(v2[u], dj), acc2);
      }
    }
  }
  const z64 s1 = block_zsum(acc1, red);
  const z64 s2 = block_zsum(acc2, red);
  if (threadIdx.x == 0) {
    for (int h = 0; h < 2; ++h) {
      const GemvOut& o = h ? o2 : o1;
      z64 out = zmul(o.alpha, h ? s2 : s1);
      if (o.w) out = zfma(o.beta, o.w[i], out);
      if (o.w2) out = zadd(out, zscale(o.w2[i], o.gamma));
      o.y[i] = out;
    }
  }
}

// The second pass of the re-formation fused with the candidates' tau: for
// row i of A = C^-1 and row i of G, the products of k_gemv2 (o1, o2, no
// design scaling) and tau[i] = sum_j A[i,j] G[i,j], all three sums in the
// order k_gemv2 and the scoring pass use (one pass over both rows instead of
// one over A and then one over A and G).
__global__ __launch_bounds__(kRowThreads) void k_gemv2_tau(const z64* A, const z64* G, int ld,
                                                           int n, GemvOut o1, GemvOut o2,
                                                           z64* tau) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int i = blockIdx.x;
  const z64* a = A + size_t(i) * ld;
  const z64* g = G + size_t(i) * ld;
  z64 acc1{0.0, 0.0}, acc2{0.0, 0.0}, acc3{0.0, 0.0};
  for (int j0 = threadIdx.x; j0 < n; j0 += kGemvUnroll * kRowThreads) {
    z64 aj[kGemvUnroll], gj[kGemvUnroll], v1[kGemvUnroll], v2[kGemvUnroll];
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int j = min(j0 + u * kRowThreads, n - 1);
      aj[u] = a[j];
      gj[u] = g[j];
      v1[u] = o1.v[j];
      v2[u] = o2.v[j];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      if (j0 + u * kRowThreads < n) {
        acc1 = zfma(aj[u], v1[u], acc1);
        acc2 = zfma(aj[u], v2[u], acc2);
        acc3 = zfma(aj[u], gj[u], acc3);
      }
    }
  }
  const z64 s1 = block_zsum(acc1, red);
  const z64 s2 = block_zsum(acc2, red);
  const z64 s3 = block_zsum(acc3, red);
  if (threadIdx.x == 0) {
    for (int h = 0; h < 2; ++h) {
      const GemvOut& o = h ? o2 : o1;
      z64 out = zmul(o.alpha, h ? s2 : s1);
      if (o.w) out = zfma(o.beta, o.w[i], out);
      if (o.w2) out = zadd(out, zscale(o.w2[i], o.gamma));
      o.y[i] = out;
    }
    tau[i] = s3;
  }
}

// x = x_b + k0^2 sum_j god[j] deps_j E[j]; writes x into the DBS state slot f
// and (on the last frequency) the objective.  One workgroup.
__global__ __launch_bounds__(kRowThreads) void k_output(ProbDev P, int f, const z64* god, z64 xb,
                                                        int last) {
  __shared__ double red[2 * (kRowThreads / 64)];
  z64 acc{0.0, 0.0};
  const double s = P.k0sq[f] * P.deps;
  const z64* E = P.E[f];
  // four entries per thread per pass, their loads issued together (same
  // summation order as one at a time)
  for (int j0 = threadIdx.x; j0 < P.nd; j0 += kGemvUnroll * kRowThreads) {
    uint32_t bj[kGemvUnroll];
    z64 gj[kGemvUnroll], ej[kGemvUnroll];
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int j = min(j0 + u * kRowThreads, P.nd - 1);
      bj[u] = P.bits[j];
      gj[u] = god[j];
      ej[u] = E[j];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u)
      if (j0 + u * kRowThreads < P.nd && bj[u]) acc = zfma(gj[u], zscale(ej[u], s), acc);
  }
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


// --------------------------------------------- unpivoted blocked inversion
// Gauss-Jordan on panels of kNpNb columns in their natural order, without
// row exchanges: for panel J with diagonal block B = M[J,J],
//     Pt[r,:] = (r in J) ? (B^-1)[r,:] : -M[r,J] B^-1,
//     M[:,j] <- D M[:,j] + Pt M[J,j]  (j outside J, D zeroes the rows J),
//     M[:,J] <- Pt,
// so after the last panel M = K^-1.  The rank-kNpNb update is one GEMM on
// the FP64 matrix cores.  For small systems the Z rows of C, [W, I] with
// W = -k2d G[Z,S], ride along below the S rows: Gauss-Jordan with the pivots
// of K turns [K; W] into [K^-1; -W K^-1], which is C^-1[:, S] (the Z columns
// of C^-1 are those of the identity), so no separate product forms
// C^-1[Z, S] (for large ones that product reads W once, cheaper than once
// per panel).  Its stability rests on the pivots of the diagonal
// blocks, which is what the system matrices of this method give (the
// self-coupling G_ii dominates each column); a zero block pivot and a probe
// residual ||K K^-1 v - v|| checked at the end flag the result in *status
// (bit 2), and the caller then inverts again with the pivot search.

// Panel 0's block inverse (the later ones run in the GEMM that forms their
// block, see k_zgemm).
template <int NB>
__global__ __launch_bounds__(256) void k_np_blockinv(const z64* S, int ld, int k0, int nb, z64* Bi,
                                                     int32_t* status) {
  np_block_inverse<NB>(S, ld, k0, nb, Bi, status);
}

// One launch per panel with two kinds of workgroup (n rows, nc columns).
// The first nrw = n / 16 form the reduced panel of rows [16 b, 16 b + 16): Pt[r][c] = (B^-1)[r - k0][c]
// for r in the panel's rows J, else -sum_q M[r][k0 + q] (B^-1)[q][c]; rows
// outside J also get the previous panel's columns finished
// (M[r][k0p + c] = Ptp[r][c], c < nbp), which the GEMM left undefined.  The
// others copy the panel's pivot rows, X[q][j] = M[k0 + q][j] (the previous
// panel's columns from Ptp, which M does not hold yet), and zero those rows
// of M.  The two kinds touch disjoint rows of M.
template <int NB>
__global__ __launch_bounds__(256) void k_np_panel(z64* S, int ld, int n, int nc, int k0, int nb,
                                                  const z64* Bi, z64* Pt, const z64* Ptp, int k0p,
                                                  int nbp, z64* X, int nrw) {
  __shared__ z64 sB[NB][NB + 1];
  __shared__ z64 sR[16][NB + 1];
  const int t = threadIdx.x;
  if (int(blockIdx.x) >= nrw) {
    const int e = int(blockIdx.x) - nrw, ncb = (nc + 255) / 256;
    const int q = e / ncb, j = (e % ncb) * 256 + t;
    if (q >= nb || j >= nc) return;
    z64* row = S + size_t(k0 + q) * ld;
    X[size_t(q) * ld + j] = (Ptp && j >= k0p && j < k0p + nbp)
                                ? Ptp[size_t(k0 + q) * kNpNb + (j - k0p)]
                                : row[j];
    row[j] = z64{0.0, 0.0};
    return;
  }
  const int r0 = blockIdx.x * 16;
  for (int e = t; e < NB * NB; e += 256) sB[e / NB][e % NB] = Bi[e];
  for (int e = t; e < 16 * NB; e += 256) {
    const int rr = e / NB, q = e % NB, r = r0 + rr;
    sR[rr][q] = (r < n && q < nb && (r < k0 || r >= k0 + nb)) ? S[size_t(r) * ld + k0 + q]
                                                              : z64{0.0, 0.0};
  }
  __syncthreads();
  const int rr = t >> 4, r = r0 + rr;
  if (r >= n) return;
  const bool inJ = r >= k0 && r < k0 + nb;
  // thread (rr, t % 16): columns t % 16 + 16 m, one read of the row entry
  // per q for its NB / 16 products
  constexpr int M = NB / 16;
  z64 acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = z64{0.0, 0.0};
  if (!inJ)
    for (int q = 0; q < nb; ++q) {
      const z64 x = sR[rr][q];
#pragma unroll
      for (int m = 0; m < M; ++m) acc[m] = zfma(x, sB[q][(t & 15) + 16 * m], acc[m]);
    }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int c = (t & 15) + 16 * m;
    z64 v{0.0, 0.0};
    if (c < nb) v = inJ ? sB[r - k0][c] : z64{-acc[m].re, -acc[m].im};
    Pt[size_t(r) * NB + c] = v;
    if (Ptp && !inJ && c < nbp) S[size_t(r) * ld + k0p + c] = Ptp[size_t(r) * NB + c];
  }
}

// The last panel's columns: M[r][k0 + c] = Pt[r][c].
__global__ __launch_bounds__(256) void k_np_last(z64* S, int ld, int n, int k0, int nb,
                                                 const z64* Pt) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int r = e / kNpNb, c = e % kNpNb;
  if (r < n && c < nb) S[size_t(r) * ld + k0 + c] = Pt[size_t(r) * kNpNb + c];
}

// The working matrix of the unpivoted inversion: row a < ns is row s_a of C
// restricted to the S columns (K), row ns + z the same for pixel z_z of Z
// (W = -k2d G[Z,S]).
__global__ __launch_bounds__(256) void k_np_gather(z64* M, const z64* G, int ld,
                                                   const int32_t* sidx, const int32_t* zidx,
                                                   int ns, double k2d) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= ns) return;
  const int gi = a < ns ? sidx[a] : zidx[a - ns];
  const z64 g = G[size_t(gi) * ld + sidx[b]];
  M[size_t(a) * ld + b] = z64{(a == b ? 1.0 : 0.0) - k2d * g.re, -k2d * g.im};
}

// C^-1 from the working matrix: C^-1[i][j] = M[rowmap[i]][pos[j]] for j in
// S, delta_ij for j in Z.  One row per blockIdx.y.
__global__ __launch_bounds__(256) void k_np_scatter(const z64* M, z64* Cinv, int ld, int nd,
                                                    const int32_t* pos, const int32_t* rowmap) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= nd) return;
  const int bj = pos[j];
  Cinv[size_t(i) * ld + j] =
      bj >= 0 ? M[size_t(rowmap[i]) * ld + bj] : z64{i == j ? 1.0 : 0.0, 0.0};
}

// piv = inv_p = identity (the unpivoted result is K^-1 itself); clears the
// residual check's maxima.
__global__ __launch_bounds__(256) void k_np_ident(int32_t* piv, int32_t* inv_p, int n,
                                                  unsigned long long* mx) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l < n) {
    piv[l] = l;
    inv_p[l] = l;
  }
  if (l < 4 * kResidParts) mx[l] = 0ull;
}

// The probe vector of the residual check: fixed, entries of modulus <= 1
// from an integer hash of the index.
__device__ __forceinline__ z64 np_probe(int b) {
  uint32_t h = uint32_t(b) * 2654435761u + 0x9E3779B9u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  const double re = double(h & 0xFFFFu) / 65536.0 - 0.5;
  const double im = double(h >> 16) / 65536.0 - 0.5;
  return z64{re, im};
}

// y = M v over the S block (M = K^-1 after the panels); one row per
// workgroup.
__global__ __launch_bounds__(kRowThreads) void k_np_resid_y(const z64* S, int ld, int n, z64* y) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int a = blockIdx.x;
  z64 acc{0.0, 0.0};
  for (int b = threadIdx.x; b < n; b += kRowThreads)
    acc = zfma(S[size_t(a) * ld + b], np_probe(b), acc);
  const z64 t = block_zsum(acc, red);
  if (threadIdx.x == 0) y[a] = t;
}

// Row a of K y - v with K = I - k2d G[S,S], the row's sum of |K_ab| and the
// largest |y_b|, into the maxima of partition a % kResidParts, mx[4 p + 0..2]
// (non-negative doubles compare as their bit patterns; the partitions keep
// the rows' atomics from queueing on three words).
__global__ __launch_bounds__(kRowThreads) void k_np_resid_k(const z64* G, int ld,
                                                            const int32_t* sidx, int n, double k2d,
                                                            const z64* y,
                                                            unsigned long long* mx) {
  __shared__ double red[2 * (kRowThreads / 64)];
  __shared__ double rmax[kRowThreads / 64], rsum[kRowThreads / 64];
  const int a = blockIdx.x, t = threadIdx.x;
  const z64* g = G + size_t(sidx[a]) * ld;
  z64 acc{0.0, 0.0};
  double ksum = 0.0, ymax = 0.0;
  // the column indices of kGemvUnroll entries first, then their loads
  // together (clamped in-range, results past the row end unused)
  for (int b0 = t; b0 < n; b0 += kGemvUnroll * kRowThreads) {
    int cb[kGemvUnroll];
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) cb[u] = sidx[min(b0 + u * kRowThreads, n - 1)];
    z64 gv[kGemvUnroll], yv[kGemvUnroll];
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      gv[u] = g[cb[u]];
      yv[u] = y[min(b0 + u * kRowThreads, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < kGemvUnroll; ++u) {
      const int b = b0 + u * kRowThreads;
      if (b < n) {
        const z64 kab{(a == b ? 1.0 : 0.0) - k2d * gv[u].re, -k2d * gv[u].im};
        acc = zfma(kab, yv[u], acc);
        ksum += sqrt(zabs2(kab));
        ymax = fmax(ymax, sqrt(zabs2(yv[u])));
      }
    }
  }
  const z64 ky = block_zsum(acc, red);
  const double s = wave_sum(ksum);
  double m = ymax;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((t & 63) == 0) {
    rsum[t >> 6] = s;
    rmax[t >> 6] = m;
  }
  __syncthreads();
  if (t == 0) {
    double ks = 0.0, ym = 0.0;
    for (int w = 0; w < kRowThreads / 64; ++w) {
      ks += rsum[w];
      ym = fmax(ym, rmax[w]);
    }
    const z64 r = zsub(ky, np_probe(a));
    unsigned long long* m = mx + 4 * (a % kResidParts);
    atomicMax(&m[0], static_cast<unsigned long long>(__double_as_longlong(sqrt(zabs2(r)))));
    atomicMax(&m[1], static_cast<unsigned long long>(__double_as_longlong(ks)));
    atomicMax(&m[2], static_cast<unsigned long long>(__double_as_longlong(ym)));
  }
}

// ||K y - v||_inf <= tol (||K||_inf ||y||_inf + ||v||_inf), else status bit 2
// (||v||_inf <= 1).
__global__ void k_np_check(const unsigned long long* mx, double tol, int32_t* status) {
  unsigned long long m0 = 0, m1 = 0, m2 = 0;
  for (int q = 0; q < kResidParts; ++q) {
    m0 = max(m0, mx[4 * q]);
    m1 = max(m1, mx[4 * q + 1]);
    m2 = max(m2, mx[4 * q + 2]);
  }
  const double res = __longlong_as_double(static_cast<long long>(m0));
  const double kn = __longlong_as_double(static_cast<long long>(m1));
  const double ym = __longlong_as_double(static_cast<long long>(m2));
  if (!(res <= tol * (kn * ym + 1.0))) atomicOr(status, 2);
}

hipError_t launch_inverse_np(z64* S, const z64* G, int ld, const int32_t* sidx, int ns,
                             int nrows, double k2d, const NpWork& w, int32_t* piv, int32_t* inv_p,
                             int32_t* status, hipStream_t s) {
  constexpr int NB = kNpNb;
  const dim3 gcols((ns + 255) / 256);
  hipLaunchKernelGGL(k_np_ident, gcols, dim3(256), 0, s, piv, inv_p, ns, w.mx);
  int cur = 0, k0p = 0, nbp = 0;
  const z64* Ptp = nullptr;
  const int nrw = (nrows + 15) / 16;
  hipLaunchKernelGGL(k_np_blockinv<NB>, dim3(1), dim3(256), 0, s, S, ld, 0, std::min(NB, ns),
                     w.Bi, status);
  for (int k0 = 0; k0 < ns; k0 += NB) {
    const int nb = std::min(NB, ns - k0);
    z64* Pt = w.Pt[cur];
    hipLaunchKernelGGL(k_np_panel<NB>, dim3(nrw + nb * int(gcols.x)), dim3(256), 0, s, S, ld,
                       nrows, ns, k0, nb, w.Bi, Pt, Ptp, k0p, nbp, w.X, nrw);
    // the update, whose workgroup of the next diagonal tile inverts it
    NpDiag dg;
    if (k0 + NB < ns) {
      dg.tile = (k0 + NB) / NB;
      dg.k0 = k0 + NB;
      dg.nb = std::min(NB, ns - k0 - NB);
      dg.Bi = w.Bi;
      dg.status = status;
    }
    hipError_t e = launch_zgemm_np(nrows, ns, nb, Pt, NB, w.X, ld, S, ld, dg, s);
    if (e != hipSuccess) return e;
    Ptp = Pt;
    k0p = k0;
    nbp = nb;
    cur ^= 1;
  }
  hipLaunchKernelGGL(k_np_last, dim3((nrows * NB + 255) / 256), dim3(256), 0, s, S, ld, nrows,
                     k0p, nbp, Ptp);
  hipLaunchKernelGGL(k_np_resid_y, dim3(ns), dim3(kRowThreads), 0, s, S, ld, ns, w.y);
  hipLaunchKernelGGL(k_np_resid_k, dim3(ns), dim3(kRowThreads), 0, s, G, ld, sidx, ns, k2d, w.y,
                     w.mx);
  hipLaunchKernelGGL(k_np_check, dim3(1), dim3(1), 0, s, w.mx, w.tol, status);
  return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
// C^-1 of C = I - k2d G diag(bits) into Cinv.  sidx/zidx/pos describe S and Z
// (pos[i] = index of i in S, or -1).  S, Pb, Pn are scratch, B1 (2 kGjNb x ld)
// too.  With np, the S block is inverted without row exchanges (status bit 2
// if that is not accurate: invert again without np); else with the pivot
// search (status bit 1 for a zero pivot).
hipError_t launch_inverse(z64* S, z64* Cinv, const z64* G, int nd, int ld, const int32_t* sidx,
                          const int32_t* zidx, const int32_t* pos, int ns, double k2d, z64* B1,
                          z64* Pb, z64* Pn, int32_t* piv, int32_t* inv_p, int32_t* used,
                          int32_t* status, int32_t* tsbuf, z64* B11inv, const NpWork* np,
                          hipStream_t s) {
  const int nz = nd - ns;
  if (ns > 0 && np) {
    // small systems carry the Z rows along (C^-1[:, S] in one pass, no
    // separate product); large ones form C^-1[Z, S] by one GEMM below, which
    // reads the Z rows once instead of once per panel
    const bool fold = ns <= kNpFoldMax;
    const int nrows = fold ? nd : ns;
    hipLaunchKernelGGL(k_np_gather, dim3((ns + 255) / 256, nrows), dim3(256), 0, s, S, G, ld,
                       sidx, zidx, ns, k2d);
    hipError_t e = launch_inverse_np(S, G, ld, sidx, ns, nrows, k2d, *np, piv, inv_p, status, s);
    if (e != hipSuccess) return e;
    if (fold) {
      hipLaunchKernelGGL(k_np_scatter, dim3((nd + 255) / 256, nd), dim3(256), 0, s, S, Cinv, ld,
                         nd, pos, np->rowmap);
      return hipGetLastError();
    }
  } else if (ns > 0) {
    // two tournament proposal lists (ids and counts) of (kGjNb + 1) ints
    // per group
    const int g0 = (ns + 63) / 64;
    int32_t* candA = tsbuf;
    int32_t* candB = candA + g0 * (kGjNb + 1);
    const dim3 gcols((ns + 255) / 256);
    // pivot rows of the even and odd panels, kept out of S during the
    // update that makes them
    z64* PRa = B1;
    z64* PRb = B1 + size_t(kGjNb) * ld;
    hipLaunchKernelGGL(k_gather_K, dim3(gcols.x, ns), dim3(256), 0, s, S, G, ld, sidx, ns, k2d,
                       used);
    hipLaunchKernelGGL(k_gj_panel_in, dim3((ns * kGjNb + 255) / 256), dim3(256), 0, s, S, ld, ns,
                       0, min(kGjNb, ns), Pb);
    for (int k0 = 0; k0 < ns; k0 += kGjNb) {
      const int nc = min(kGjNb, ns - k0);
      if (ns <= kGeppRows) {
        // partial pivoting over every row in one workgroup
        launch_tsel_gepp(Pb, ns, k0, nc, nullptr, nullptr, 0, ns, piv, used, B11inv, status, s);
      } else {
        // tournament levels on the chip (64-row groups, then merges of four
        // groups' proposals) until one workgroup can take every proposal
        int g = (ns + 63) / 64;
        int32_t* cand = candA;
        int32_t* cnt = candA + g * kGjNb;
        hipLaunchKernelGGL(k_tsel_wave, dim3(g), dim3(64), 0, s, Pb, ns, nc, used,
                           static_cast<const int32_t*>(nullptr),
                           static_cast<const int32_t*>(nullptr), 0, cand, cnt);
        while (g * kGjNb > kGeppRows) {
          const int ng = (g + 3) / 4;
          int32_t* ocand = (cand == candA) ? candB : candA;
          int32_t* ocnt = ocand + ng * kGjNb;
          hipLaunchKernelGGL(k_tsel_wave, dim3(ng), dim3(64), 0, s, Pb, ns, nc, used, cand, cnt,
                             g, ocand, ocnt);
          cand = ocand;
          cnt = ocnt;
          g = ng;
        }
        launch_tsel_gepp(Pb, ns, k0, nc, cand, cnt, g, g * kGjNb, piv, used, B11inv, status, s);
      }
      const bool odd = (k0 / kGjNb) & 1;
      if (ns >= kUpdBigFrom)
        hipLaunchKernelGGL(k_gj_update<kUpdRowsBig>,
                           dim3((ns + 63) / 64, (ns + kUpdRowsBig - 1) / kUpdRowsBig), dim3(256),
                           0, s, S, ld, ns, k0, nc, used, piv, B11inv, Pb, odd ? PRa : PRb,
                           odd ? PRb : PRa, Pn);
      else
        hipLaunchKernelGGL(k_gj_update<kUpdRows>,
                           dim3((ns + 63) / 64, (ns + kUpdRows - 1) / kUpdRows), dim3(256), 0, s,
                           S, ld, ns, k0, nc, used, piv, B11inv, Pb, odd ? PRa : PRb,
                           odd ? PRb : PRa, Pn);
      z64* t = Pb;
      Pb = Pn;
      Pn = t;
    }
    const int klast = (ns - 1) / kGjNb * kGjNb;
    hipLaunchKernelGGL(k_gj_rows_back, dim3(gcols.x, ns - klast), dim3(256), 0, s, S, ld, ns,
                       klast, ns - klast, piv, ((klast / kGjNb) & 1) ? PRb : PRa);
    hipLaunchKernelGGL(k_gj_invperm, dim3(gcols.x), dim3(256), 0, s, piv, inv_p, ns);
  }
  const dim3 grow((nd + 255) / 256, nd);
  hipLaunchKernelGGL(k_scatter_inverse, grow, dim3(256), 0, s, S, Cinv, ld, nd, pos, piv, inv_p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ns > 0 && nz > 0) {
    // C^-1[Z, S] = k2d G[Z, S] C^-1[S, S] on the FP64 matrix cores
    GemmIdx ix;
    ix.ra = zidx;
    ix.ca = sidx;
    ix.rb = sidx;
    ix.cb = sidx;
    ix.rc = zidx;
    ix.cc = sidx;
    // split K so that the grid covers the chip (about two workgroups of
    // 64 x 64 outputs per CU); the partial products go to S, free once
    // K^-1 has been scattered (splits * nz * ns <= nd * ld)
    const int tiles = ((nz + 63) / 64) * ((ns + 63) / 64);
    int splits = (512 + tiles - 1) / tiles;
    splits = std::max(1, std::min(splits, 4));
    while (splits > 1 && size_t(splits) * nz * ns > size_t(nd) * ld) --splits;
    e = launch_zgemm_ix(nz, ns, ns, G, ld, Cinv, ld, false, Cinv, ld, ix, z64{k2d, 0.0},
                        z64{0.0, 0.0}, splits, splits > 1 ? S : nullptr, s);
  }
  return e;
}

hipError_t launch_gemv(const z64* A, int ld, int n, const z64* v, const uint8_t* bits, double ds,
                       z64 alpha, z64 beta, const z64* w, double gamma, const z64* w2, z64* y,
                       hipStream_t s, z32* A32) {
  hipLaunchKernelGGL(k_gemv, dim3(n), dim3(kRowThreads), 0, s, A, ld, n, v, bits, ds, alpha, beta,
                     w, gamma, w2, y, A32);
  return hipGetLastError();
}

hipError_t launch_gemv2(const z64* A, int ld, int n, const uint8_t* bits, double ds,
                        const GemvOut& o1, const GemvOut& o2, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv2, dim3(n), dim3(kRowThreads), 0, s, A, ld, n, bits, ds, o1, o2);
  return hipGetLastError();
}

hipError_t launch_gemv2_tau(const z64* A, const z64* G, int ld, int n, const GemvOut& o1,
                            const GemvOut& o2, z64* tau, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv2_tau, dim3(n), dim3(kRowThreads), 0, s, A, G, ld, n, o1, o2, tau);
  return hipGetLastError();
}

hipError_t launch_output(const ProbDev& P, int f, const z64* god, z64 xb, int last,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(1), dim3(kRowThreads), 0, s, P, f, god, xb, last);
  return hipGetLastError();
}

}  // namespace pngf
