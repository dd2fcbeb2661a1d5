// Mixed-precision support kernels of libpngf (gfx950): the complex-FP32 copy
// of C0^-1, the rank-k Woodbury fold on the FP32 matrix cores, and the
// measurement of the FP32 score error that sets the decision band.  The
// per-step kernel of the mixed search is k_mixed_step (step_kernels.hip).
//
// Between FP64 re-inversions the inverse is held as
//     C^-1 = C0^-1 + sum_k alpha_k p_k q_k^T            (eq. lru_woodbury, M = 1,
//                                                       applied lazily)
// with C0^-1 and G in complex FP32.  Accepting pixel m needs
//     p = C^-1 g_m = C0^-1 g_m + sum_k alpha_k p_k (q_k . g_m),
//     q = C^-1[m,:] = C0^-1[m,:] + sum_k alpha_k p_k[m] q_k ,
// and by reciprocity (C^-1 G is symmetric) q_k . g_m = p_k[m], so both use the
// coefficients c_k = alpha_k p_k[m].  The candidate scores of the new state
// follow from tau_i += alpha p_i (G q)_i; E, R', tau and x stay FP64 vectors.
// Per accept the matrices are streamed once each in FP32: 2 N_d^2 x 8 B.
#include "dev_state.h"

namespace pngf {

__device__ __forceinline__ z64 up(z32 a) { return {double(a.re), double(a.im)}; }
__device__ __forceinline__ z32 down(z64 a) { return {float(a.re), float(a.im)}; }

// C0^-1 <- complex FP32 copy of a complex FP64 matrix (nd x ld rows).
__global__ __launch_bounds__(256) void k_to_c64(const z64* src, z32* dst, int nd, int ld) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < nd) dst[size_t(i) * ld + j] = down(src[size_t(i) * ld + j]);
}

// Rank-k Woodbury fold C0^-1 += sum_k alpha_k p_k q_k^T on the FP32 matrix
// cores (v_mfma_f32_16x16x4f32).  A complex product is four real ones:
// Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br with A = alpha P (N_d x k) and
// B = Q^T (k x N_d).  A workgroup of 4 waves owns a 32x32 tile, one 16x16
// tile per wave.  Operand layouts (16x16x4): lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r holds D[4(l/16)+r][l%16].
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_fold(ProbDev P, int f, int kp) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i0 = blockIdx.y * 32 + (wid >> 1) * 16;
  const int j0 = blockIdx.x * 32 + (wid & 1) * 16;
  const int ld = P.ld, nd = P.nd;
  const z32* Pp = P.Pp[f];
  const z32* Qp = P.Qp[f];
  const z64* al = P.alph[f];
  f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
  const int ai = i0 + (lane & 15);   // A row (< ld: padded rows hold 0)
  const int bj = j0 + (lane & 15);   // B column
  for (int k0 = 0; k0 < kp; k0 += 4) {
    const int k = k0 + (lane >> 4);
    float ar = 0.f, aim = 0.f, br = 0.f, bim = 0.f;
    if (k < kp) {
      const z64 a = zmul(al[k], up(Pp[size_t(k) * ld + ai]));
      ar = float(a.re);
      aim = float(a.im);
      const z32 b = Qp[size_t(k) * ld + bj];
      br = b.re;
      bim = b.im;
    }
    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-aim, bim, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bim, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(aim, br, ci, 0, 0, 0);
  }
  z32* C = P.C0[f];
  const int j = j0 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * (lane >> 4) + r;
    if (i < nd && j < nd) {
      z32 v = C[size_t(i) * ld + j];
      v.re += cr[r];
      v.im += ci[r];
      C[size_t(i) * ld + j] = v;
    }
  }
}

// max_i |df64_i - df32_i| / bound_i over all candidates: the FP32 error of the
// scores just before an FP64 re-inversion, relative to their bound.
// out[0] = the measurement; out[1] = *status (nullable) as a double, so that
// one read brings both to the host; bandp (nullable) receives the band the
// measurement sets, min(1e-2, max(1e-6, 100 m)) when m is finite.
// gate (nullable): the measurement is skipped while *gate is 0.
__global__ __launch_bounds__(256) void k_band_measure(const double* df32, const double* bnd32,
                                                      const double* df64, int nd, double* out,
                                                      const int32_t* status, double* bandp,
                                                      const int32_t* gate) {
  __shared__ double red[4];
  if (gate && *gate == 0) return;
  double mx = 0.0;
  for (int i = threadIdx.x; i < nd; i += 256) {
    const double b = bnd32[i];
    if (b > 0.0) mx = fmax(mx, fabs(df64[i] - df32[i]) / b);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    out[0] = m;
    out[1] = status ? double(*status) : 0.0;
    if (bandp && isfinite(m)) *bandp = fmin(1e-2, fmax(1e-6, 100.0 * m));
  }
}

// The device-side start of a refresh that the host queues behind a batch of
// steps before it has read the batch's end state (one workgroup):
//  * an odd number of updates since the last normalization leaves the
//    current E, R', tau and design in the B buffers: they are copied to the
//    A buffers (the state's flip count back to 0), so that the refresh and
//    the next batch read the A set;
//  * the pixels whose bit differs from the design bref of C^-1, ascending,
//    with the scales k0^2 (+-delta eps) of each frequency (dS[f kpad + c]),
//    padded to kpad entries with pixel 0 and scale 0 (zero columns of the
//    block-Woodbury panel); bref becomes the current design (that of C^-1
//    once the update is done);
//  * wk[0] = their count (above kpad the capacitance kernel reports it),
//    wk[1] = 1 when the scores are FP32 results to be measured (the state is
//    not exact);
//  * the state and key slots as a segment starts (what k_segment_start does
//    with a panel reset; nothing before the rescoring reads them).
constexpr int kPrepThreads = 1024;

__global__ __launch_bounds__(kPrepThreads) void k_wood_prep(ProbDev P, uint8_t* bref, int kpad,
                                                            int32_t* dF, double* dS, int32_t* wk) {
  uint32_t* keys = P.keys;
  constexpr int kW = kPrepThreads / 64;
  __shared__ int wcnt[kW];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  DbsState* st = P.st;
  const int odd = st->flips & 1;
  if (odd) {
    for (int i = tid; i < P.nd; i += kPrepThreads) {
      for (int f = 0; f < P.nfreq; ++f) {
        P.E[f][i] = P.EB[f][i];
        P.Rp[f][i] = P.RpB[f][i];
        P.tau[f][i] = P.tauB[f][i];
      }
      P.bits[i] = P.bitsB[i];
    }
  }
  if (tid == 0) base = 0;
  __syncthreads();
  for (int i0 = 0; i0 < P.nd; i0 += kPrepThreads) {
    const int i = i0 + tid;
    const uint8_t b = i < P.nd ? P.bits[i] : 0;   // this thread copied bits[i]
    const bool d = i < P.nd && b != bref[i];
    if (d) bref[i] = b;   // the design of C^-1 once the update is done
    const uint64_t bal = __ballot(d);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int v = 0; v < w; ++v) off += wcnt[v];
    if (d && off + pre < kpad) {
      const int c = off + pre;
      dF[c] = i;
      const double delta = b ? P.deps : -P.deps;
      for (int f = 0; f < P.nfreq; ++f) dS[size_t(f) * kpad + c] = P.k0sq[f] * delta;
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int v = 0; v < kW; ++v) t += wcnt[v];
      base += t;
    }
    __syncthreads();
  }
  const int k = base;
  for (int c = k + tid; c < kpad; c += kPrepThreads) {
    dF[c] = 0;
    for (int f = 0; f < P.nfreq; ++f) dS[size_t(f) * kpad + c] = 0.0;
  }
  if (tid < 6) keys[tid] = kNoKey;
  if (tid == 0) {
    wk[0] = k;
    wk[1] = st->exact ? 0 : 1;
    // the start of the next segment: no pending update, an empty panel,
    // exact scores (those the refresh computes), every key slot empty
    st->m = -1;
    st->kpanel = 0;
    st->n_since = 0;
    st->exact = 1;
    st->need_refresh = 0;
    st->flips = 0;
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_to_c64(const z64* src, z32* dst, int nd, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_to_c64, dim3((nd + 255) / 256, nd), dim3(256), 0, s, src, dst, nd, ld);
  return hipGetLastError();
}

hipError_t launch_fold(const ProbDev& P, int f, int kp, hipStream_t s) {
  if (kp <= 0) return hipSuccess;
  const int t = (P.nd + 31) / 32;
  hipLaunchKernelGGL(k_fold, dim3(t, t), dim3(256), 0, s, P, f, kp);
  return hipGetLastError();
}

hipError_t launch_band_measure(const double* df32, const double* bnd32, const double* df64,
                               int nd, double* out, const int32_t* status, hipStream_t s,
                               double* bandp, const int32_t* gate) {
  hipLaunchKernelGGL(k_band_measure, dim3(1), dim3(256), 0, s, df32, bnd32, df64, nd, out, status,
                     bandp, gate);
  return hipGetLastError();
}

hipError_t launch_wood_prep(const ProbDev& P, uint8_t* bref, int kpad, int32_t* dF,
                            double* dS, int32_t* wk, hipStream_t s) {
  hipLaunchKernelGGL(k_wood_prep, dim3(1), dim3(kPrepThreads), 0, s, P, bref, kpad, dF, dS, wk);
  return hipGetLastError();
}

}  // namespace pngf
