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
// A panel of kGjNb columns picks its pivot rows by tournament pivoting
// (Grigori-Demmel-Xiang CALU): groups of 64 rows, one group per wave, each
// propose kGjNb rows by partial-pivoting elimination in registers; the
// proposals of four groups form the next level's group until one remains
// (the first levels one wave per workgroup across the chip, the last ones in
// one workgroup); the winners' block B11 is inverted and every row is reduced
// independently, giving the Gauss-Jordan panel [-B01 B11^-1; B11^-1;
// -B21 B11^-1].  Every column outside the panel then gets the rank-kGjNb
// update M[r,j] = (r pivot of this panel ? 0 : M[r,j]) + P[r,:] B1[:,j] with
// B1 the panel's pivot rows before the update (the reduction of the panel
// rows happens inside the update's workgroups, and the new pivot rows wait
// in a side buffer until the next panel's update, so no workgroup reads a
// row another one writes).  On gfx950 the FP64
// matrix-core rate equals the FP64 vector rate (78.6 TFLOP/s), and at this
// panel width the update is HBM-bound, so it runs on the vector ALUs.
#include <utility>

#include "dev_state.h"

namespace pngf {

hipError_t launch_zgemm_ix(int M, int N, int K, const z64* A, int lda, const z64* B, int ldb,
                           bool transb, z64* C, int ldc, const GemmIdx& ix, z64 alpha, z64 beta,
                           int splits, z64* work, hipStream_t s, int* nz_out = nullptr);

constexpr int kGjNb = 16;
constexpr int kUpdRows = 16;      // rows per update workgroup (small systems)
constexpr int kUpdRowsBig = 64;   // ... from kUpdBigFrom pivot rows on: the pivot rows'
constexpr int kUpdBigFrom = 2048; // values and the panel factors are shared by more rows

// K[a][b] = delta_ab - k2d G[s_a][s_b]; clears the pivot marks.
__global__ __launch_bounds__(256) void k_gather_K(z64* K, const z64* G, int ld, const int32_t* sidx,
                                                  int ns, double k2d, int32_t* used,
                                                  int32_t* arrived) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (a == 0 && b == 0) *arrived = 0;
  if (b >= ns) return;
  const z64 g = G[size_t(sidx[a]) * ld + sidx[b]];
  K[size_t(a) * ld + b] = z64{(a == b ? 1.0 : 0.0) - k2d * g.re, -k2d * g.im};
  if (a == 0) used[b] = 0;
}

// Panel columns [k0, k0+ncols) gathered into a contiguous n x kGjNb buffer.
__global__ __launch_bounds__(256) void k_gj_panel_in(const z64* S, int ld, int n, int k0,
                                                     int ncols, z64* Pb) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int r = e / kGjNb, c = e % kGjNb;
  if (r < n) Pb[e] = (c < ncols) ? S[size_t(r) * ld + k0 + c] : z64{0.0, 0.0};
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
__device__ __forceinline__ bool wave_tournament(const z64* Pb, int ncols, int row, int lane,
                                                int* out, int* cnt) {
  z32 a[kGjNb];
#pragma unroll
  for (int c = 0; c < kGjNb; ++c) {
    z32 v{0.f, 0.f};
    if (row >= 0 && c < ncols) {
      const z64 x = Pb[size_t(row) * kGjNb + c];
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

// Gauss-Jordan column C of [B11 | I] held one column per lane (lane j holds
// column j, rows in registers): the pivot row is every lane's own register C,
// the factors column C come from lane C by readlane.
template <int C>
__device__ __forceinline__ void gj_lane_column(z64 (&w)[kGjNb]) {
  const z64 pv{lane_d(w[C].re, C), lane_d(w[C].im, C)};
  const z64 inv = (zabs2(pv) > 0.0) ? zdiv(z64{1.0, 0.0}, pv) : z64{0.0, 0.0};
  const z64 prow = zmul(w[C], inv);
#pragma unroll
  for (int i = 0; i < kGjNb; ++i) {
    if (i == C) continue;
    const z64 f{lane_d(w[i].re, C), lane_d(w[i].im, C)};
    w[i] = zsub(w[i], zmul(f, prow));
  }
  w[C] = prow;
}

template <int... Cs>
__device__ __forceinline__ void gj_lane_columns(z64 (&w)[kGjNb],
                                                std::integer_sequence<int, Cs...>) {
  (gj_lane_column<Cs>(w), ...);
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
  wave_tournament(Pb, ncols, row, lane, cand + g * kGjNb, cnt + g);
}

// Device-coherent accesses of the proposal lists that workgroups of one
// launch exchange (written through to memory, read around the caches).
__device__ __forceinline__ void st_coh(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coh(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0 of the workgroup that holds the winners (prop[0..nsel), in pivot
// order): piv, used and B11^-1 (inverted in FP64, one column per lane), and
// a zero pivot of the final level flagged in *status.
__device__ __forceinline__ void tsel_finish(const z64* Pb, int k0, int ncols, const int* win,
                                            int nsel, bool zero, int lane, int32_t* piv,
                                            int32_t* used, z64* B11inv, int32_t* status) {
  if (zero && lane == 0) atomicOr(status, 1);
  const int j = lane;
  z64 w[kGjNb];
#pragma unroll
  for (int r = 0; r < kGjNb; ++r) {
    z64 v{0.0, 0.0};
    if (j < kGjNb) {
      if (r < nsel && j < ncols) v = Pb[size_t(win[r]) * kGjNb + j];
      else if (r == j) v = z64{1.0, 0.0};       // padding of a ragged panel
    } else if (j - kGjNb == r) {
      v = z64{1.0, 0.0};
    }
    w[r] = v;
  }
  gj_lane_columns(w, std::make_integer_sequence<int, kGjNb>{});
  if (j >= kGjNb && j < 2 * kGjNb)
#pragma unroll
    for (int r = 0; r < kGjNb; ++r) B11inv[r * kGjNb + (j - kGjNb)] = w[r];
  if (lane < nsel) {
    const int rw = win[lane];
    piv[k0 + lane] = rw;
    used[rw] = k0 + lane + 1;
  }
}

// The rest of a panel's tournament in one workgroup of nw = blockDim/64 <= 16
// waves.  Its first level is either level 0 itself (gcand null, n <= 64 nw:
// one group of 64 rows per wave) or a merge of the ngin <= 4 nw groups that
// k_tsel_l0 proposed (four per wave).  Each further level merges the
// proposals of four groups in one wave, with a barrier between levels, until
// wave 0 holds the winners.  Wave 0 then writes piv, used and B11^-1
// (inverted in FP64, one column per lane), and flags a zero pivot of the
// final level in *status.
__global__ __launch_bounds__(1024) void k_tsel_wg(const z64* Pb, int n, int k0, int ncols,
                                                  const int32_t* gcand, const int32_t* gcnt,
                                                  int ngin, int32_t* piv, int32_t* used,
                                                  z64* B11inv, int32_t* status) {
  __shared__ int prop[2][16 * kGjNb];
  __shared__ int pcnt[2][16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  int groups = int(blockDim.x) >> 6;
  int row = -1;
  if (gcand == nullptr) {
    row = wid * 64 + lane;
    if (row >= n || used[row]) row = -1;
  } else {
    const int grp = wid * 4 + lane / kGjNb, u = lane % kGjNb;
    if (grp < ngin && u < gcnt[grp]) row = gcand[grp * kGjNb + u];
  }
  bool zero = wave_tournament(Pb, ncols, row, lane, &prop[0][wid * kGjNb], &pcnt[0][wid]);
  int cur = 0;
  while (groups > 1) {
    __syncthreads();
    const int ng = (groups + 3) / 4;
    if (wid < ng) {
      const int grp = wid * 4 + lane / kGjNb, u = lane % kGjNb;
      const int r = (grp < groups && u < pcnt[cur][grp]) ? prop[cur][grp * kGjNb + u] : -1;
      zero = wave_tournament(Pb, ncols, r, lane, &prop[cur ^ 1][wid * kGjNb], &pcnt[cur ^ 1][wid]);
    }
    cur ^= 1;
    groups = ng;
  }
  __syncthreads();
  if (wid != 0) return;
  tsel_finish(Pb, k0, ncols, &prop[cur][0], pcnt[cur][0], zero, lane, piv, used, B11inv, status);
}


// A panel's whole tournament in one launch for 64 < n <= 4096: workgroup g
// (four waves, one per SIMD) runs level 0 on rows [256g, 256g + 256), one
// group of 64 rows per wave, and wave 0 merges its four groups; the
// proposals go to cand/cnt through device-coherent stores, and the last
// workgroup to count itself in on *arrived (each waits for its stores first)
// merges every workgroup's proposals, four groups per wave, and finishes.  It
// also puts *arrived back to zero for the next panel.
__global__ __launch_bounds__(256) void k_tsel_fused(const z64* Pb, int n, int k0, int ncols,
                                                    int32_t* cand, int32_t* cnt,
                                                    int32_t* arrived, int32_t* piv,
                                                    int32_t* used, z64* B11inv,
                                                    int32_t* status) {
  __shared__ int prop[2][4 * kGjNb];
  __shared__ int pcnt[2][4];
  __shared__ int s_last;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6, g = blockIdx.x;
  const int G = gridDim.x;
  int row = g * 256 + wid * 64 + lane;
  if (row >= n || used[row]) row = -1;
  wave_tournament(Pb, ncols, row, lane, &prop[0][wid * kGjNb], &pcnt[0][wid]);
  __syncthreads();
  bool zero = false;
  if (wid == 0) {
    const int grp = lane / kGjNb, u = lane % kGjNb;
    const int r = (u < pcnt[0][grp]) ? prop[0][grp * kGjNb + u] : -1;
    zero = wave_tournament(Pb, ncols, r, lane, &prop[1][0], &pcnt[1][0]);
    if (G > 1) {
      const int c = pcnt[1][0];
      if (lane < c) st_coh(cand + g * kGjNb + lane, prop[1][lane]);
      if (lane == 0) st_coh(cnt + g, c);
      __builtin_amdgcn_s_waitcnt(0);
      if (lane == 0) s_last = (atomicAdd(arrived, 1) == G - 1) ? 1 : 0;
    }
  }
  __syncthreads();
  if (G == 1) {
    // one workgroup: its merge is the final level
    if (wid == 0)
      tsel_finish(Pb, k0, ncols, &prop[1][0], pcnt[1][0], zero, lane, piv, used, B11inv,
                  status);
    return;
  }
  if (!s_last) return;
  // the last workgroup: merge the G <= 16 proposal lists, four per wave
  int groups = (G + 3) / 4;
  {
    const int grp = wid * 4 + lane / kGjNb, u = lane % kGjNb;
    int r = -1;
    if (wid < groups && grp < G && u < ld_coh(cnt + grp)) r = ld_coh(cand + grp * kGjNb + u);
    if (wid < groups)
      zero = wave_tournament(Pb, ncols, r, lane, &prop[0][wid * kGjNb], &pcnt[0][wid]);
  }
  int cur = 0;
  while (groups > 1) {
    __syncthreads();
    const int ng = (groups + 3) / 4;
    if (wid < ng) {
      const int grp = wid * 4 + lane / kGjNb, u = lane % kGjNb;
      const int r = (grp < groups && u < pcnt[cur][grp]) ? prop[cur][grp * kGjNb + u] : -1;
      zero = wave_tournament(Pb, ncols, r, lane, &prop[cur ^ 1][wid * kGjNb], &pcnt[cur ^ 1][wid]);
    }
    cur ^= 1;
    groups = ng;
  }
  __syncthreads();
  if (wid != 0) return;
  if (lane == 0) st_coh(arrived, 0);
  tsel_finish(Pb, k0, ncols, &prop[cur][0], pcnt[cur][0], zero, lane, piv, used, B11inv, status);
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
    const int rr = e / kGjNb, c = e % kGjNb;
    const int r = r0 + rr;
    R[rr][c] = (r < n && c < ncols) ? Pb[size_t(r) * kGjNb + c] : z64{0.0, 0.0};
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
    if (in_next) Pn[size_t(r0 + rr) * kGjNb + (j - nxt)] = acc;
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
__global__ __launch_bounds__(kRowThreads) void k_gemv(const z64* A, int ld, int n, const z64* v,
                                                      const uint8_t* bits, double ds, z64 alpha,
                                                      z64 beta, const z64* w, double gamma,
                                                      const z64* w2, z64* y, z32* A32) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int i = blockIdx.x;
  const z64* a = A + size_t(i) * ld;
  z64 acc{0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += kRowThreads) {
    z64 vj = v[j];
    if (bits) vj = zscale(vj, bits[j] ? ds : 0.0);
    const z64 aij = a[j];
    if (A32) A32[size_t(i) * ld + j] = z32{float(aij.re), float(aij.im)};
    acc = zfma(aij, vj, acc);
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
  for (int j = threadIdx.x; j < n; j += kRowThreads) {
    const double dj = bits ? (bits[j] ? ds : 0.0) : 1.0;
    const z64 aj = a[j];
    acc1 = zfma(aj, zscale(o1.v[j], dj), acc1);
    acc2 = zfma(aj, zscale(o2.v[j], dj), acc2);
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
// C^-1 of C = I - k2d G diag(bits) into Cinv.  sidx/zidx/pos describe S and Z
// (pos[i] = index of i in S, or -1).  S, Pb, Pn are scratch, B1 (2 kGjNb x ld)
// too.
hipError_t launch_inverse(z64* S, z64* Cinv, const z64* G, int nd, int ld, const int32_t* sidx,
                          const int32_t* zidx, const int32_t* pos, int ns, double k2d, z64* B1,
                          z64* Pb, z64* Pn, int32_t* piv, int32_t* inv_p, int32_t* used,
                          int32_t* status, int32_t* tsbuf, z64* B11inv, hipStream_t s) {
  const int nz = nd - ns;
  if (ns > 0) {
    // the arrival count of the fused tournament, then two proposal lists
    // (ids and counts) of (kGjNb + 1) ints per group
    const int g0 = (ns + 63) / 64;
    int32_t* arrived = tsbuf;
    int32_t* candA = tsbuf + 64;
    int32_t* candB = candA + g0 * (kGjNb + 1);
    const dim3 gcols((ns + 255) / 256);
    // pivot rows of the even and odd panels, kept out of S during the
    // update that makes them
    z64* PRa = B1;
    z64* PRb = B1 + size_t(kGjNb) * ld;
    hipLaunchKernelGGL(k_gather_K, dim3(gcols.x, ns), dim3(256), 0, s, S, G, ld, sidx, ns, k2d,
                       used, arrived);
    hipLaunchKernelGGL(k_gj_panel_in, dim3((ns * kGjNb + 255) / 256), dim3(256), 0, s, S, ld, ns,
                       0, min(kGjNb, ns), Pb);
    for (int k0 = 0; k0 < ns; k0 += kGjNb) {
      const int nc = min(kGjNb, ns - k0);
      if (ns <= 64) {
        hipLaunchKernelGGL(k_tsel_wg, dim3(1), dim3(64), 0, s, Pb, ns, k0, nc,
                           static_cast<const int32_t*>(nullptr),
                           static_cast<const int32_t*>(nullptr), 0, piv, used, B11inv, status);
      } else if (ns <= 16 * 256) {
        const int g = (ns + 255) / 256;
        hipLaunchKernelGGL(k_tsel_fused, dim3(g), dim3(256), 0, s, Pb, ns, k0, nc, candA,
                           candA + g * kGjNb, arrived, piv, used, B11inv, status);
      } else {
        // level 0, then merge levels on the chip until one workgroup's
        // sixteen waves can merge the rest (<= 64 groups)
        int g = (ns + 63) / 64;
        int32_t* cand = candA;
        int32_t* cnt = candA + g * kGjNb;
        hipLaunchKernelGGL(k_tsel_wave, dim3(g), dim3(64), 0, s, Pb, ns, nc, used,
                           static_cast<const int32_t*>(nullptr),
                           static_cast<const int32_t*>(nullptr), 0, cand, cnt);
        while (g > 64) {
          const int ng = (g + 3) / 4;
          int32_t* ocand = (cand == candA) ? candB : candA;
          int32_t* ocnt = ocand + ng * kGjNb;
          hipLaunchKernelGGL(k_tsel_wave, dim3(ng), dim3(64), 0, s, Pb, ns, nc, used, cand, cnt,
                             g, ocand, ocnt);
          cand = ocand;
          cnt = ocnt;
          g = ng;
        }
        hipLaunchKernelGGL(k_tsel_wg, dim3(1), dim3(64 * ((g + 3) / 4)), 0, s, Pb, ns, k0, nc,
                           cand, cnt, g, piv, used, B11inv, status);
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

hipError_t launch_output(const ProbDev& P, int f, const z64* god, z64 xb, int last,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(1), dim3(kRowThreads), 0, s, P, f, god, xb, last);
  return hipGetLastError();
}

}  // namespace pngf
