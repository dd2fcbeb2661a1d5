// Mixed-precision DBS kernels of libpngf (gfx950): complex-FP32 matrices with
// a deferred Sherman-Morrison panel, FP64 state vectors, an error band that
// sends borderline decisions to the FP64 state, and the rank-k Woodbury fold
// on the FP32 matrix cores.
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

__device__ __forceinline__ uint32_t mkey(const ProbDev& P, const DbsState* st, int i) {
  const int s = st->cursor_s;
  if (s >= st->n_sweeps) return kNoKey;
  const int pos = P.rank[size_t(s) * P.nd + i];
  if (pos >= st->cursor_pos) return uint32_t(pos);
  if (s + 1 < st->n_sweeps) return uint32_t(P.nd + P.rank[size_t(s + 1) * P.nd + i]);
  return kNoKey;
}

// Select for the mixed path: a candidate inside the error band ahead of every
// sure improvement stops the search for an FP64 re-inversion (need_refresh=2);
// so does the periodic interval or a full panel (need_refresh=1).  Otherwise
// as the FP64 select: decode the first improving position, advance the cursor,
// form alpha and the panel coefficients c_k = alpha_k p_k[m].
__global__ __launch_bounds__(kRowThreads) void k_mixed_select(ProbDev P) {
  __shared__ int s_m, s_slot;
  DbsState* st = P.st;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int m = -1;
    const int nd = P.nd;
    if (!st->done && !st->need_refresh) {
      const uint32_t key = st->key, km = st->key_maybe;
      if (st->n_acc >= P.max_acc || st->cursor_s >= st->n_sweeps) {
        st->done = 1;
        st->converged = 0;
      } else if (!st->exact && km != kNoKey && (key == kNoKey || km < key)) {
        st->need_refresh = 2;
      } else if (!st->exact && ((P.k_refresh > 0 && st->n_since >= P.k_refresh) ||
                                st->kpanel >= P.kcap)) {
        st->need_refresh = 1;
      } else {
        const int s = st->cursor_s, c = st->cursor_pos, ns = st->n_sweeps;
        if (key == kNoKey) {
          // every candidate is surely not improving (no band hit either)
          const bool next = (c > 0) && (s + 1 < ns);
          st->attempts += (nd - c) + (next ? nd : 0);
          st->converged = (c == 0) || next;
          st->sweeps = s + 1 + (next ? 1 : 0);
          st->done = 1;
        } else {
          int s2 = s, pos = int(key);
          if (int(key) >= nd) {
            s2 = s + 1;
            pos = int(key) - nd;
            st->attempts += (nd - c) + pos + 1;
          } else {
            st->attempts += pos - c + 1;
          }
          m = P.perm[size_t(s2) * nd + pos];
          st->sweeps = s2 + 1;
          if (pos + 1 < nd) {
            st->cursor_s = s2;
            st->cursor_pos = pos + 1;
          } else {
            st->cursor_s = s2 + 1;
            st->cursor_pos = 0;
          }
        }
      }
    }
    if (m >= 0 || st->done) {
      st->key = kNoKey;
      st->key_maybe = kNoKey;
    }
    int slot = -1;
    if (m >= 0) {
      slot = st->kpanel;
      const double delta = P.bits[m] ? -P.deps : P.deps;
      double fnew = 0.0;
      for (int f = 0; f < P.nfreq; ++f) {
        const double kd = P.k0sq[f] * delta;
        const z64 tau = P.tau[f][m];
        const z64 den = {1.0 - kd * tau.re, -kd * tau.im};
        const z64 alpha = zdiv(z64{kd, 0.0}, den);
        const z64 Em = P.E[f][m], Rpm = P.Rp[f][m];
        st->alpha[f] = alpha;
        st->Em[f] = Em;
        st->Rpm[f] = Rpm;
        P.alph[f][slot] = alpha;
        const z64 x = zfma(zmul(alpha, Em), Rpm, st->x[f]);
        st->x[f] = x;
        fnew += P.coef[f] * zabs2(x);
      }
      P.bits[m] ^= 1;
      st->f = fnew;
      P.log_pix[st->n_acc] = m;
      P.log_f[st->n_acc] = fnew;
      st->n_acc += 1;
      st->n_since += 1;
      st->kpanel = slot + 1;
      st->exact = 0;
    }
    st->m = m;
    st->kslot = slot;
    s_m = m;
    s_slot = slot;
  }
  __syncthreads();
  const int m = s_m, slot = s_slot;
  if (m < 0) return;
  for (int f = 0; f < P.nfreq; ++f)
    for (int k = tid; k < slot; k += kRowThreads)
      P.pcoef[f][k] = zmul(P.alph[f][k], up(P.Pp[f][size_t(k) * P.ld + m]));
}

// q = C0^-1[m,:] + sum_k c_k q_k, stored as the new panel q slot.
__global__ __launch_bounds__(256) void k_mixed_q(ProbDev P) {
  const DbsState* st = P.st;
  const int m = st->m;
  if (m < 0) return;
  const int slot = st->kslot;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= P.nd) return;
  for (int f = 0; f < P.nfreq; ++f) {
    z64 acc = up(P.C0[f][size_t(m) * P.ld + j]);
    for (int k = 0; k < slot; ++k)
      acc = zfma(P.pcoef[f][k], up(P.Qp[f][size_t(k) * P.ld + j]), acc);
    P.Qp[f][size_t(slot) * P.ld + j] = down(acc);
  }
}

__device__ __forceinline__ void block_fsum4(float& a, float& b, float& c, float& d, float* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  a = wave_sumf(a);
  b = wave_sumf(b);
  c = wave_sumf(c);
  d = wave_sumf(d);
  if (lane == 0) {
    red[4 * wid] = a;
    red[4 * wid + 1] = b;
    red[4 * wid + 2] = c;
    red[4 * wid + 3] = d;
  }
  __syncthreads();
  a = b = c = d = 0.f;
  for (int w = 0; w < nw; ++w) {
    a += red[4 * w];
    b += red[4 * w + 1];
    c += red[4 * w + 2];
    d += red[4 * w + 3];
  }
  __syncthreads();
}

// Row i: p_i = C0^-1[i,:] . g_m + sum_k c_k p_k[i] and s_i = G[i,:] . q
// (FP32 accumulation); appends p_i to the panel; E, R', tau updated in FP64;
// candidate i of the new state scored with its error bound.
template <int NPL>
__global__ __launch_bounds__(kRowThreads) void k_mixed_accept(ProbDev P) {
  __shared__ float red[4 * (kRowThreads / 64)];
  const DbsState* st = P.st;
  const int m = st->m;
  if (m < 0) return;
  const int slot = st->kslot;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const double delta = P.bits[i] ? -P.deps : P.deps;
  double df = 0.0, bnd = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    const z32* c0 = P.C0[f] + size_t(i) * P.ld;
    const z32* gm = P.G32[f] + size_t(m) * P.ld;
    const z32* gi = P.G32[f] + size_t(i) * P.ld;
    const z32* q = P.Qp[f] + size_t(slot) * P.ld;
    float pr = 0.f, pi = 0.f, sr = 0.f, si = 0.f;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) {
        const z32 a = c0[j], b = gm[j], g = gi[j], u = q[j];
        pr = fmaf(a.re, b.re, fmaf(-a.im, b.im, pr));
        pi = fmaf(a.re, b.im, fmaf(a.im, b.re, pi));
        sr = fmaf(g.re, u.re, fmaf(-g.im, u.im, sr));
        si = fmaf(g.re, u.im, fmaf(g.im, u.re, si));
      }
    }
    if (tid < slot) {
      const z64 c = P.pcoef[f][tid];
      const z32 pk = P.Pp[f][size_t(tid) * P.ld + i];
      pr += float(c.re * pk.re - c.im * pk.im);
      pi += float(c.re * pk.im + c.im * pk.re);
    }
    block_fsum4(pr, pi, sr, si, red);
    if (tid == 0) {
      const z64 p = {double(pr), double(pi)}, s = {double(sr), double(si)};
      P.Pp[f][size_t(slot) * P.ld + i] = z32{pr, pi};
      const z64 ap = zmul(st->alpha[f], p);
      const z64 Ei = zadd(P.E[f][i], zmul(ap, st->Em[f]));
      const z64 Rpi = zadd(P.Rp[f][i], zmul(ap, st->Rpm[f]));
      const z64 tau = zadd(P.tau[f][i], zmul(ap, s));
      P.E[f][i] = Ei;
      P.Rp[f][i] = Rpi;
      P.tau[f][i] = tau;
      const double kd = P.k0sq[f] * delta;
      const z64 den = {1.0 - kd * tau.re, -kd * tau.im};
      const z64 dx = zdiv(zscale(zmul(Ei, Rpi), kd), den);
      const z64 x = st->x[f];
      const double adx = sqrt(zabs2(dx));
      df += P.coef[f] * (2.0 * (x.re * dx.re + x.im * dx.im) + adx * adx);
      bnd += P.coef[f] * (2.0 * sqrt(zabs2(x)) * adx + adx * adx);
    }
  }
  if (tid == 0) {
    P.df32[i] = df;
    P.dfb[i] = bnd;
    const double margin = df - st->eta * st->f;
    const double band = P.band * bnd;
    if (margin >= -band) {
      const uint32_t k = mkey(P, st, i);
      if (k != kNoKey) atomicMin(margin > band ? &P.st->key : &P.st->key_maybe, k);
    }
  }
}

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
__global__ __launch_bounds__(256) void k_band_measure(const double* df32, const double* bnd32,
                                                      const double* df64, int nd, double* out) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int i = threadIdx.x; i < nd; i += 256) {
    const double b = bnd32[i];
    if (b > 0.0) mx = fmax(mx, fabs(df64[i] - df32[i]) / b);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ------------------------------------------------------------------ launchers
hipError_t launch_mixed_select(const ProbDev& P, hipStream_t s) {
  hipLaunchKernelGGL(k_mixed_select, dim3(1), dim3(kRowThreads), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_mixed_q(const ProbDev& P, hipStream_t s) {
  hipLaunchKernelGGL(k_mixed_q, dim3((P.nd + 255) / 256), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_mixed_accept(const ProbDev& P, int npl, hipStream_t s) {
  switch (npl) {
    case 1: hipLaunchKernelGGL(k_mixed_accept<1>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    case 2: hipLaunchKernelGGL(k_mixed_accept<2>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    case 4: hipLaunchKernelGGL(k_mixed_accept<4>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    case 8: hipLaunchKernelGGL(k_mixed_accept<8>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    case 16: hipLaunchKernelGGL(k_mixed_accept<16>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    case 32: hipLaunchKernelGGL(k_mixed_accept<32>, dim3(P.nd), dim3(kRowThreads), 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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
                               int nd, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_band_measure, dim3(1), dim3(256), 0, s, df32, bnd32, df64, nd, out);
  return hipGetLastError();
}

}  // namespace pngf
