// The diagonal-block inverse of the unpivoted blocked FP64 inversion, shared
// by its own kernel (the first panel) and the GEMM that forms every later
// block (which inverts it as soon as its tile is done).
#pragma once

#include "dev_state.h"

namespace pngf {

// 1/z in FP64: the hardware reciprocal estimate of |z|^2 refined by two
// Newton steps (each squares the relative error), 0 for z = 0.  Shorter
// than the IEEE division sequence on the pivot chains below.
__device__ __forceinline__ z64 zrecip_newton(z64 z) {
  const double d = z.re * z.re + z.im * z.im;
  double x = __builtin_amdgcn_rcp(d);
  x = fma(x, fma(-d, x, 1.0), x);
  x = fma(x, fma(-d, x, 1.0), x);
  if (!(d > 0.0)) x = 0.0;
  return z64{z.re * x, -z.im * x};
}

// Workgroup barrier that orders LDS accesses only, for kernels whose waves
// exchange nothing else through it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The block inverse: B^-1 of M[k0..k0+nb, k0..k0+nb] (identity-padded to
// NB x NB) by in-place Gauss-Jordan without pivoting, in one workgroup of
// 256 threads, thread (ti, tj) = (t / 16, t % 16) holding the T x T tile of
// rows T ti .., columns T tj .. in registers.  Step C: the pivot column's
// entries of a thread's rows come from lane C / T of its own 16-lane row
// (ds_bpermute), the pivot row through LDS (two buffers by parity, one
// barrier per step).  The tile columns are a loop, and only the four steps
// within one are unrolled: straight-line code for all 64 steps would not fit
// the instruction cache.
__device__ __forceinline__ z64 lane_bperm(z64 v, int src) {
  const int addr = src << 2;
  const long long r = __double_as_longlong(v.re), i = __double_as_longlong(v.im);
  const uint32_t r0 = __builtin_amdgcn_ds_bpermute(addr, int(uint32_t(r)));
  const uint32_t r1 = __builtin_amdgcn_ds_bpermute(addr, int(uint32_t(uint64_t(r) >> 32)));
  const uint32_t i0 = __builtin_amdgcn_ds_bpermute(addr, int(uint32_t(i)));
  const uint32_t i1 = __builtin_amdgcn_ds_bpermute(addr, int(uint32_t(uint64_t(i) >> 32)));
  return z64{__longlong_as_double(static_cast<long long>((uint64_t(r1) << 32) | r0)),
             __longlong_as_double(static_cast<long long>((uint64_t(i1) << 32) | i0))};
}

// Step C = T oc + RC of the block inverse (RC known at compile time, so the
// pivot column's and row's registers are named directly).
template <int NB, int RC>
__device__ __forceinline__ void np_block_step(z64 (&a)[NB / 16][NB / 16], int oc, int ti, int tj,
                                              int lane, z64 (&rowbuf)[2][NB], bool& bad) {
  constexpr int T = NB / 16;
  constexpr int par = RC & 1;   // C = T oc + RC has the parity of RC (T even)
  const int C = T * oc + RC;
  const int src = (lane & 48) | oc;
  z64 col[T];
#pragma unroll
  for (int r = 0; r < T; ++r) col[r] = lane_bperm(a[r][RC], src);
  if (ti == oc) {
#pragma unroll
    for (int k = 0; k < T; ++k) rowbuf[par][T * tj + k] = a[RC][k];
  }
  lds_barrier();
  z64 u[T];
#pragma unroll
  for (int k = 0; k < T; ++k) u[k] = rowbuf[par][T * tj + k];
  const z64 pv = rowbuf[par][C];
  if (!(pv.re * pv.re + pv.im * pv.im > 1e-280)) bad = true;
  const z64 inv = zrecip_newton(pv);
  // a <- alpha_i a' + beta_i u'_j with a' = 0 and u' = 1 in the pivot
  // column, alpha = 0 and beta = 1/p for the pivot row, alpha = 1 and
  // beta = -a_iC/p elsewhere: the pivot row scaled, the pivot column -a_iC/p
  // (1/p at the pivot), every other entry reduced
  const bool pcol = tj == oc;
  if (pcol) u[RC] = z64{1.0, 0.0};
#pragma unroll
  for (int r = 0; r < T; ++r) {
    const bool prow = ti == oc && r == RC;
    const z64 f = zmul(col[r], inv);
    const z64 beta = prow ? inv : z64{-f.re, -f.im};
#pragma unroll
    for (int k = 0; k < T; ++k) {
      z64 x = a[r][k];
      if (prow || (pcol && k == RC)) x = z64{0.0, 0.0};
      a[r][k] = zfma(beta, u[k], x);
    }
  }
}

template <int NB>
__device__ __forceinline__ void np_block_inverse(const z64* S, int ld, int k0, int nb, z64* Bi,
                                                 int32_t* status) {
  constexpr int T = NB / 16;
  static_assert(T == 4, "four steps per tile column");
  __shared__ z64 rowbuf[2][NB];
  const int t = threadIdx.x, ti = t >> 4, tj = t & 15, lane = t & 63;
  z64 a[T][T];
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int i = T * ti + r, j = T * tj + k;
      a[r][k] = (i < nb && j < nb) ? S[size_t(k0 + i) * ld + k0 + j]
                                   : z64{i == j ? 1.0 : 0.0, 0.0};
    }
  bool bad = false;
#pragma unroll 1
  for (int oc = 0; oc < 16; ++oc) {
    np_block_step<NB, 0>(a, oc, ti, tj, lane, rowbuf, bad);
    np_block_step<NB, 1>(a, oc, ti, tj, lane, rowbuf, bad);
    np_block_step<NB, 2>(a, oc, ti, tj, lane, rowbuf, bad);
    np_block_step<NB, 3>(a, oc, ti, tj, lane, rowbuf, bad);
  }
#pragma unroll
  for (int r = 0; r < T; ++r)
#pragma unroll
    for (int k = 0; k < T; ++k) Bi[(T * ti + r) * NB + T * tj + k] = a[r][k];
  if (bad && threadIdx.x == 0) atomicOr(status, 2);
}

}  // namespace pngf
