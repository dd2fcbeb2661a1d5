// Multi-pixel flips (tiles of M pixels flipped together) for libpngf (gfx950):
// the exact rank-M score of every tile from the current FP64 state.
//
// Field form, K = diag(k0^2 deps) over the design: C = I - G K, T = C^-1 G
// (complex symmetric), E = C^-1 b, R' = G_OD (I + K T).  Flipping the pixel
// set S changes K by D = diag(d_S), d_i = k0^2 delta_i, i.e. C by the rank-M
// term U V with U = -G[:,S] D, V = I[S,:] (eq. lru_dcn).  The Woodbury
// identity (eq. lru_woodbury) with the capacitance I + V C^-1 U = I - T_SS D
// gives, with W = D (I - T_SS D)^-1,
//     x' = x + R'[S]^T W E[S]                                  (eq. lru_eobj_rs)
//     C^-1 += T[:,S] W C^-1[S,:],  E += T[:,S] W E[S],  R' += (R'[S]^T W) T[S,:].
// Scoring needs only the M x M block T_SS = C^-1[S,:] G[:,S] = C^-1[S,:] G[S,:]^T
// (reciprocity): M^2 dot products of length N_d per tile, which is one read of
// C^-1 and G for all tiles together.  The accept is the FP64 block-Woodbury
// update on the matrix cores (the same kernels as the mixed form's refresh).
//
// Two kernels per frequency:
//   k_tile_partial: workgroup (tile t, K slice s) streams the tile's rows of
//     C^-1 and G over its column slice through LDS in chunks of kTileKc
//     (register prefetch of the next chunk); thread (ti, tj) accumulates the
//     RB x RB entries (ti + 16a, tj + 16b) of the slice's partial T_SS.
//     Slicing K gives ntiles x KS workgroups, so the chain of chunk loads of
//     one workgroup is short and the whole chip streams.
//   k_tile_solve: workgroup t sums the slices, solves (I - T_SS D) y = E[S]
//     by Gauss-Jordan with partial pivoting in LDS (pivot rows recorded, not
//     swapped: two barriers per column), and adds
//     dx = sum_i R'[s_i] d_i y_i,  df_f = coef (2 Re(conj(x) dx) + |dx|^2)
//     to the tile's score.  A singular capacitance gives NaN (never accepted).
#include "dev_state.h"

namespace pngf {

constexpr int kTileThreads = 256;
constexpr int kTileKc = 32;  // columns per LDS chunk

// Chunk element u of this thread: matrix u / HALF (0: C^-1, 1: G) with
// HALF = PER / 2, local element e = tid + (u % HALF) kTileThreads of that
// matrix's MR x kTileKc chunk: row e / kTileKc of the tile, column
// k0 + e % kTileKc (< kend).
template <int MR, int PER>
__device__ __forceinline__ void tile_fetch(z64 (&reg)[PER], const z64* Cf, const z64* Gf,
                                           const int* pix, int ld, int kend, int k0, int tid) {
  constexpr int HALF = PER / 2;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + (u % HALF) * kTileThreads;
    const int r = e / kTileKc, c = e % kTileKc;
    const int p = pix[r];
    const z64* src = (u < HALF ? Cf : Gf) + size_t(p < 0 ? 0 : p) * ld + k0 + c;
    double re = 0.0, im = 0.0;
    if (p >= 0 && k0 + c < kend) {
      re = src->re;
      im = src->im;
    }
    reg[u] = z64{re, im};
  }
}

// Tile pixel ids (padded rows -1) into LDS; returns the tile's pixel count.
template <int MR>
__device__ __forceinline__ int tile_load_pix(const int32_t* tiles, int t, int m, int* pix) {
  const int tid = threadIdx.x;
  if (tid < MR) pix[tid] = tid < m ? tiles[size_t(t) * m + tid] : -1;
  __syncthreads();
  int c = 0;
  for (int i = 0; i < MR; ++i) c += pix[i] >= 0;
  return c;
}

template <int RB>
__global__ __launch_bounds__(kTileThreads) void k_tile_partial(ProbDev P, const int32_t* tiles,
                                                               int ntiles, int m, int f, int ks,
                                                               z64* part) {
  constexpr int MR = 16 * RB;
  constexpr int CH = MR * (kTileKc + 1);
  constexpr int PER = 2 * MR * kTileKc / kTileThreads;
  static_assert(MR * kTileKc % kTileThreads == 0, "chunk must split evenly over the threads");
  __shared__ z64 As[CH];
  __shared__ z64 Bs[CH];
  __shared__ int pix[MR];
  const int t = blockIdx.x, s = blockIdx.y;
  if (t >= ntiles || s >= ks) return;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  tile_load_pix<MR>(tiles, t, m, pix);
  // column slice of this workgroup, whole chunks
  const int nchunk = (P.nd + kTileKc - 1) / kTileKc;
  const int c0 = int((int64_t(nchunk) * s) / ks), c1 = int((int64_t(nchunk) * (s + 1)) / ks);
  const int kbeg = c0 * kTileKc, kend = min(P.nd, c1 * kTileKc);
  const z64* Cf = P.Cinv[f];
  const z64* Gf = P.G[f];
  z64 acc[RB][RB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[a][b] = z64{0.0, 0.0};
  z64 reg[PER];
  if (kbeg < kend) tile_fetch<MR, PER>(reg, Cf, Gf, pix, P.ld, kend, kbeg, tid);
  for (int k0 = kbeg; k0 < kend; k0 += kTileKc) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + (u % (PER / 2)) * kTileThreads;
      const int r = e / kTileKc, c = e % kTileKc;
      if (u < PER / 2) As[r * (kTileKc + 1) + c] = reg[u];
      else Bs[r * (kTileKc + 1) + c] = reg[u];
    }
    __syncthreads();
    if (k0 + kTileKc < kend) tile_fetch<MR, PER>(reg, Cf, Gf, pix, P.ld, kend, k0 + kTileKc, tid);
#pragma unroll 4
    for (int c = 0; c < kTileKc; ++c) {
      z64 av[RB], bv[RB];
#pragma unroll
      for (int a = 0; a < RB; ++a) av[a] = As[(ti + 16 * a) * (kTileKc + 1) + c];
#pragma unroll
      for (int b = 0; b < RB; ++b) bv[b] = Bs[(tj + 16 * b) * (kTileKc + 1) + c];
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          acc[a][b].re += av[a].re * bv[b].re - av[a].im * bv[b].im;
          acc[a][b].im += av[a].re * bv[b].im + av[a].im * bv[b].re;
        }
    }
  }
  z64* out = part + (size_t(t) * ks + s) * MR * MR;
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) out[(ti + 16 * a) * MR + tj + 16 * b] = acc[a][b];
}

template <int RB>
__global__ __launch_bounds__(kTileThreads) void k_tile_solve(ProbDev P, const int32_t* tiles,
                                                             int ntiles, int m, int f, int ks,
                                                             const z64* part, int first,
                                                             double* out) {
  constexpr int MR = 16 * RB;
  constexpr int LDA = MR + 1;
  __shared__ z64 Ax[MR * LDA];
  __shared__ int pix[MR];
  __shared__ double dsc[MR];
  __shared__ int rowof[MR];   // physical row of the pivot of each column
  __shared__ int used[MR];
  __shared__ int s_bad;
  const int t = blockIdx.x;
  if (t >= ntiles) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ti = tid >> 4, tj = tid & 15;
  if (tid == 0) s_bad = 0;
  if (tid < MR) used[tid] = 0;
  const int mt = tile_load_pix<MR>(tiles, t, m, pix);
  if (tid < MR) {
    const int p = pix[tid];
    dsc[tid] = p >= 0 ? P.k0sq[f] * (P.bits[p] ? -P.deps : P.deps) : 0.0;
  }
  __syncthreads();
  // augmented system [I - T_SS D | E_S] over the tile's rows
  const z64* pb = part + size_t(t) * ks * MR * MR;
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      if (i < mt && j < mt) {
        z64 v{0.0, 0.0};
#pragma unroll 8
        for (int s = 0; s < ks; ++s) v = zadd(v, pb[size_t(s) * MR * MR + i * MR + j]);
        const double dj = dsc[j];
        v = z64{-v.re * dj, -v.im * dj};
        if (i == j) v.re += 1.0;
        Ax[i * LDA + j] = v;
      }
    }
  if (tid < mt) Ax[tid * LDA + mt] = P.E[f][pix[tid]];
  __syncthreads();
  // Gauss-Jordan with partial pivoting; pivot rows are recorded instead of
  // swapped, and every thread forms its own row's factor, so a column costs
  // two barriers.
  for (int c = 0; c < mt; ++c) {
    if (wid == 0) {
      double best = -1.0;
      int bi = MR;
      for (int i = lane; i < mt; i += 64) {
        if (used[i]) continue;
        const double v = zabs2(Ax[i * LDA + c]);
        if (v > best || (v == best && i < bi)) { best = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) {
        if (!(best > 0.0) || bi >= mt) {
          s_bad = 1;
          bi = 0;
          for (int i = 0; i < mt; ++i)
            if (!used[i]) { bi = i; break; }
        }
        rowof[c] = bi;
        used[bi] = 1;
      }
    }
    __syncthreads();
    const int pr = rowof[c];
    const z64 piv = Ax[pr * LDA + c];
    const bool ok = zabs2(piv) > 0.0;
    const int w = mt - c;  // columns c+1 .. mt (rhs included)
    for (int e = tid; e < mt * w; e += kTileThreads) {
      const int i = e / w, j = c + 1 + e % w;
      if (i != pr && ok) {
        const z64 fac = zdiv(Ax[i * LDA + c], piv);
        Ax[i * LDA + j] = zsub(Ax[i * LDA + j], zmul(fac, Ax[pr * LDA + j]));
      }
    }
    __syncthreads();
  }
  // dx = sum_c R'[s_c] d_c y_c with y_c = rhs / pivot of column c's pivot row
  if (wid == 0) {
    z64 dx{0.0, 0.0};
    for (int cc = lane; cc < mt; cc += 64) {
      const int r = rowof[cc];
      const z64 piv = Ax[r * LDA + cc];
      const z64 y = zabs2(piv) > 0.0 ? zdiv(Ax[r * LDA + mt], piv) : z64{0.0, 0.0};
      dx = zadd(dx, zscale(zmul(P.Rp[f][pix[cc]], y), dsc[cc]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dx.re += __shfl_xor(dx.re, o);
      dx.im += __shfl_xor(dx.im, o);
    }
    if (lane == 0) {
      const z64 x = P.st->x[f];
      const double df = P.coef[f] * (2.0 * (x.re * dx.re + x.im * dx.im) + zabs2(dx));
      const double prev = first ? 0.0 : out[t];
      out[t] = s_bad ? __builtin_nan("") : prev + df;
    }
  }
}

// part: workspace of at least ntiles * ks * (16 RB)^2 complex entries.
template <int RB>
static hipError_t tile_score_rb(const ProbDev& P, const int32_t* tiles, int ntiles, int m, int ks,
                                z64* part, double* out, hipStream_t s) {
  for (int f = 0; f < P.nfreq; ++f) {
    hipLaunchKernelGGL(k_tile_partial<RB>, dim3(ntiles, ks), dim3(kTileThreads), 0, s, P, tiles,
                       ntiles, m, f, ks, part);
    hipLaunchKernelGGL(k_tile_solve<RB>, dim3(ntiles), dim3(kTileThreads), 0, s, P, tiles, ntiles,
                       m, f, ks, part, f == 0 ? 1 : 0, out);
  }
  return hipGetLastError();
}

int tile_rows(int m) { return m <= 16 ? 16 : (m <= 32 ? 32 : 64); }

hipError_t launch_tile_score(const ProbDev& P, const int32_t* tiles, int ntiles, int m, int ks,
                             z64* part, double* out, hipStream_t s) {
  if (ks < 1) return hipErrorInvalidValue;
  if (m <= 16) return tile_score_rb<1>(P, tiles, ntiles, m, ks, part, out, s);
  if (m <= 32) return tile_score_rb<2>(P, tiles, ntiles, m, ks, part, out, s);
  if (m <= 64) return tile_score_rb<4>(P, tiles, ntiles, m, ks, part, out, s);
  return hipErrorInvalidValue;
}

}  // namespace pngf
