// FP64 plain-path kernels of libpngf (gfx950): candidate scoring, select,
// and the fused Sherman-Morrison accept + rescore pass.
//
// Field form of the PNGF system (Supplementary Note 4, C = I + Y G, written
// for fields): C = I - k0^2 G diag(deps), E = C^-1 b, and the output row
// R' = G_OD (I + k0^2 diag(deps) C^-1 G), so that x = x_b + k0^2 G_OD D E.
// Flipping pixel m by delta changes C by the rank-1 term -k0^2 delta g_m e_m^T
// (eq. lru_dcn with M = 1).  With tau_m = (C^-1 G)[m,m] and
// den = 1 - k0^2 delta tau_m the candidate output is
//     x' = x + (k0^2 delta E[m] / den) R'[m]                  (eq. lru_eobj_rs)
// and accepting it updates (eq. lru_woodbury with M = 1, alpha = k0^2 delta/den)
//     p = C^-1 g_m,  q = C^-1[m,:],  C^-1 += alpha p q^T,
//     E += alpha E[m] p,  R' += alpha R'[m] p,  x += alpha E[m] R'[m].
// G is symmetric (reciprocity), so tau_i = sum_j C^-1[i,j] G[i,j] and
// g_m = G[m,:]: every operand is streamed along rows (coalesced).
//
// Bandwidth plan: one 256-thread workgroup per matrix row; lanes hold the row
// of C^-1 in registers between the two reductions of the fused pass, so HBM
// sees one read and one write of C^-1 and one read of G per accept
// (3 N_d^2 x 16 B); g_m and q are re-read by every row from L2.
#include "dev_state.h"

namespace pngf {

__device__ __forceinline__ uint32_t cand_key(const ProbDev& P, const DbsState* st, int i) {
  const int s = st->cursor_s;
  if (s >= st->n_sweeps) return kNoKey;
  const int pos = P.rank[size_t(s) * P.nd + i];
  if (pos >= st->cursor_pos) return pack_key(pos, i);
  if (s + 1 < st->n_sweeps) return pack_key(P.nd + P.rank[size_t(s + 1) * P.nd + i], i);
  return kNoKey;
}

// Objective change of flipping pixel i given tau_f(i) (lane-0 epilogue).
__device__ __forceinline__ double flip_df(const ProbDev& P, const DbsState* st, int f,
                                          z64 tau, z64 Ei, z64 Rpi, double delta) {
  const double kd = P.k0sq[f] * delta;
  const z64 den = {1.0 - kd * tau.re, -kd * tau.im};
  const z64 dx = zdiv(zscale(zmul(Ei, Rpi), kd), den);
  const z64 x = st->x[f];
  return P.coef[f] * (2.0 * (x.re * dx.re + x.im * dx.im) + zabs2(dx));
}

// K1: tau_i = sum_j C^-1[i,j] G[i,j] for each candidate row and its exact
// objective change; with keyp, improving candidates compete for the smallest
// visiting key.
template <int NPL>
__global__ __launch_bounds__(kRowThreads) void k_score_rows(ProbDev P, const int32_t* cand,
                                                            int ncand, uint32_t* keyp) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int r = blockIdx.x;
  if (r >= ncand) return;
  const int i = cand ? cand[r] : r;
  const int tid = threadIdx.x;
  const DbsState* st = P.st;
  const double delta = P.bits[i] ? -P.deps : P.deps;
  double df = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    const z64* C = P.Cinv[f] + size_t(i) * P.ld;
    const z64* Gi = P.G[f] + size_t(i) * P.ld;
    // every load issued before the first product (an entry past the row
    // loads a clamped address and is not summed): one memory round trip
    z64 cv[NPL], gv[NPL];
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = min(tid + t * kRowThreads, P.nd - 1);
      cv[t] = C[j];
      gv[t] = Gi[j];
    }
    z64 acc{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t)
      if (tid + t * kRowThreads < P.nd) acc = zfma(cv[t], gv[t], acc);
    const z64 tau = block_zsum(acc, red);
    if (tid == 0) {
      P.tau[f][i] = tau;
      df += flip_df(P, st, f, tau, P.E[f][i], P.Rp[f][i], delta);
    }
  }
  if (tid == 0) {
    P.df[r] = df;
    if (keyp && df > st->eta * st->f) {
      const uint32_t k = cand_key(P, st, i);
      if (k != kNoKey) atomicMin(keyp, k);
    }
  }
}

// The scoring epilogue of every pixel from tau, E and R' already formed (by
// the fused re-formation pass): the same objective change and key as
// k_score_rows, one thread per pixel, the keys of a wave reduced to one
// atomic.
__global__ __launch_bounds__(256) void k_score_tail(ProbDev P, uint32_t* keyp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const DbsState* st = P.st;
  uint32_t k = kNoKey;
  if (i < P.nd) {
    const double delta = P.bits[i] ? -P.deps : P.deps;
    double df = 0.0;
    for (int f = 0; f < P.nfreq; ++f)
      df += flip_df(P, st, f, P.tau[f][i], P.E[f][i], P.Rp[f][i], delta);
    P.df[i] = df;
    if (keyp && df > st->eta * st->f) k = cand_key(P, st, i);
  }
  // wave minimum of the keys (the maximum of their complements)
  k = ~wave_max_u32(~k);
  if (keyp && (threadIdx.x & 63) == 0 && k != kNoKey) atomicMin(keyp, k);
}

// The end of a single-frequency refresh in one workgroup, three passes in
// one launch: x = x_b + k0^2 sum_j god_j deps_j E_j and f (the first 256
// threads, in k_output's order), then every pixel's objective change and key
// from tau, E and R' (as k_score_tail), and, with bandp, the error band from
// the largest |df64 - df32| / bound over the pixels (as k_band_measure: out
// = {max, 0}, band = clamp(100 max) when gate is unset or nonzero).
constexpr int kTailThreads = 1024;
__global__ __launch_bounds__(kTailThreads) void k_refresh_tail(ProbDev P, const z64* god, z64 xb,
                                                               uint32_t* keyp, const double* df32,
                                                               const double* dfb, double* out,
                                                               double* bandp, const int32_t* gate) {
  __shared__ double red[2 * (kTailThreads / 64)];
  const int tid = threadIdx.x;
  DbsState* st = P.st;
  z64 acc{0.0, 0.0};
  if (tid < kRowThreads) {
    const double s = P.k0sq[0] * P.deps;
    const z64* E = P.E[0];
    for (int j0 = tid; j0 < P.nd; j0 += 4 * kRowThreads) {
      uint32_t bj[4];
      z64 gj[4], ej[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = min(j0 + u * kRowThreads, P.nd - 1);
        bj[u] = P.bits[j];
        gj[u] = god[j];
        ej[u] = E[j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j0 + u * kRowThreads < P.nd && bj[u]) acc = zfma(gj[u], zscale(ej[u], s), acc);
    }
  }
  // the other waves add zeros after the first four's sums (the same result)
  const z64 t = block_zsum(acc, red);
  if (tid == 0) {
    // f in the operation order k_output is compiled to (explicit fused
    // multiply-adds, so that both give the same bits)
    const z64 x = zadd(xb, t);
    st->x[0] = x;
    st->f = fma(P.coef[0], fma(x.re, x.re, x.im * x.im), 0.0);
  }
  __syncthreads();
  const bool meas = bandp && (!gate || *gate != 0);
  uint32_t kmin = kNoKey;
  double mx = 0.0;
  for (int i = tid; i < P.nd; i += kTailThreads) {
    const double delta = P.bits[i] ? -P.deps : P.deps;
    double df = 0.0;
    df += flip_df(P, st, 0, P.tau[0][i], P.E[0][i], P.Rp[0][i], delta);
    P.df[i] = df;
    if (keyp && df > st->eta * st->f) kmin = min(kmin, cand_key(P, st, i));
    if (meas) {
      const double b = dfb[i];
      if (b > 0.0) mx = fmax(mx, fabs(df - df32[i]) / b);
    }
  }
  kmin = ~wave_max_u32(~kmin);
  if (keyp && (tid & 63) == 0 && kmin != kNoKey) atomicMin(keyp, kmin);
  if (meas) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < kTailThreads / 64; ++w) m = fmax(m, red[w]);
      out[0] = m;
      out[1] = 0.0;
      if (isfinite(m)) *bandp = fmin(1e-2, fmax(1e-6, 100.0 * m));
    }
  }
}

// K2: select the first improving candidate in visiting order (the minimum
// key), advance the cursor, form the update scalars of the accepted flip and
// stage q = C^-1[m,:].  forced >= 0 accepts that pixel instead.
__global__ __launch_bounds__(kRowThreads) void k_select_prep(ProbDev P, int forced) {
  __shared__ int s_m;
  DbsState* st = P.st;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int m = -1;
    const int nd = P.nd;
    if (!st->done) {
      if (forced >= 0) {
        m = forced;
      } else if (st->n_acc >= P.max_acc || st->cursor_s >= st->n_sweeps) {
        st->done = 1;
        st->converged = 0;
      } else {
        const uint32_t key = st->key;
        const int s = st->cursor_s, c = st->cursor_pos, ns = st->n_sweeps;
        if (key == kNoKey) {
          // Nothing improves at this state: the rest of this sweep is visited
          // and, if this sweep kept something, one more full sweep.
          const bool next = (c > 0) && (s + 1 < ns);
          st->attempts += (nd - c) + (next ? nd : 0);
          st->converged = (c == 0) || next;
          st->sweeps = s + 1 + (next ? 1 : 0);
          st->done = 1;
        } else {
          int s2 = s, pos = key_vis(key);
          if (pos >= nd) {
            s2 = s + 1;
            pos -= nd;
            st->attempts += (nd - c) + pos + 1;
          } else {
            st->attempts += pos - c + 1;
          }
          m = key_pixel(key);
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
    st->key = kNoKey;
    if (m >= 0) {
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
        const z64 x = zfma(zmul(alpha, Em), Rpm, st->x[f]);
        st->x[f] = x;
        fnew += P.coef[f] * zabs2(x);
      }
      P.bits[m] ^= 1;
      st->f = fnew;
      if (forced < 0) {
        P.log_pix[st->n_acc] = m;
        P.log_f[st->n_acc] = fnew;
        st->n_acc += 1;
      }
    }
    st->m = m;
    s_m = m;
  }
  __syncthreads();
  const int m = s_m;
  if (m < 0) return;
  for (int f = 0; f < P.nfreq; ++f) {
    const z64* src = P.Cinv[f] + size_t(m) * P.ld;
    z64* dst = P.q[f];
    for (int j = tid; j < P.nd; j += kRowThreads) dst[j] = src[j];
  }
}

// K3: fused accept + rescore.  Row i: p_i = C^-1[i,:] . g_m, then
// C^-1[i,:] += alpha p_i q, E[i], R'[i] updated, and tau_i of the new state
// from the updated row and G[i,:]; the new state's candidate i is scored.
template <int NPL>
__global__ __launch_bounds__(kRowThreads) void k_accept_rescore(ProbDev P) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const DbsState* st = P.st;
  const int m = st->m;
  if (m < 0) return;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const double delta = P.bits[i] ? -P.deps : P.deps;
  double df = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    z64* C = P.Cinv[f] + size_t(i) * P.ld;
    const z64* gm = P.G[f] + size_t(m) * P.ld;
    const z64* Gi = P.G[f] + size_t(i) * P.ld;
    const z64* q = P.q[f];
    z64 row[NPL];
    z64 acc{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) {
        row[t] = C[j];
        acc = zfma(row[t], gm[j], acc);
      }
    }
    const z64 p = block_zsum(acc, red);
    const z64 ap = zmul(st->alpha[f], p);
    acc = z64{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) {
        row[t] = zfma(ap, q[j], row[t]);
        C[j] = row[t];
        acc = zfma(row[t], Gi[j], acc);
      }
    }
    const z64 tau = block_zsum(acc, red);
    if (tid == 0) {
      const z64 Ei = zadd(P.E[f][i], zmul(ap, st->Em[f]));
      const z64 Rpi = zadd(P.Rp[f][i], zmul(ap, st->Rpm[f]));
      P.E[f][i] = Ei;
      P.Rp[f][i] = Rpi;
      P.tau[f][i] = tau;
      df += flip_df(P, st, f, tau, Ei, Rpi, delta);
    }
  }
  if (tid == 0) {
    P.df[i] = df;
    if (df > st->eta * st->f) {
      const uint32_t k = cand_key(P, st, i);
      if (k != kNoKey) atomicMin(&P.st->key, k);
    }
  }
}

// Accept only (no rescore): row i of C^-1 += alpha p_i q with
// p_i = C^-1[i,:] . g_m, and E, R' updated; 2 N_d^2 x 16 B per accept.  Used
// by the learned search, which scores only the proposed candidates exactly.
template <int NPL>
__global__ __launch_bounds__(kRowThreads) void k_accept_only(ProbDev P) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const DbsState* st = P.st;
  const int m = st->m;
  if (m < 0) return;
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  for (int f = 0; f < P.nfreq; ++f) {
    z64* C = P.Cinv[f] + size_t(i) * P.ld;
    const z64* gm = P.G[f] + size_t(m) * P.ld;
    const z64* q = P.q[f];
    z64 row[NPL];
    z64 acc{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) {
        row[t] = C[j];
        acc = zfma(row[t], gm[j], acc);
      }
    }
    const z64 p = block_zsum(acc, red);
    const z64 ap = zmul(st->alpha[f], p);
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) C[j] = zfma(ap, q[j], row[t]);
    }
    if (tid == 0) {
      P.E[f][i] = zadd(P.E[f][i], zmul(ap, st->Em[f]));
      P.Rp[f][i] = zadd(P.Rp[f][i], zmul(ap, st->Rpm[f]));
    }
  }
}

// Best improving candidate among df[0..n): out = cand[r] (or r) maximizing
// df with df > eta f, or -1.  One workgroup.
__global__ __launch_bounds__(1024) void k_pick_best(const double* df, const int32_t* cand, int n,
                                                   const DbsState* st, int32_t* out) {
  __shared__ double bv[16];
  __shared__ int bi[16];
  const double thr = st->eta * st->f;
  double best = -INFINITY;
  int idx = -1;
  for (int r = threadIdx.x; r < n; r += 1024)
    if (df[r] > thr && df[r] > best) { best = df[r]; idx = r; }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ob > best || (ob == best && oi >= 0 && (idx < 0 || oi < idx))) { best = ob; idx = oi; }
  }
  if ((threadIdx.x & 63) == 0) { bv[threadIdx.x >> 6] = best; bi[threadIdx.x >> 6] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bv[0];
    int id = bi[0];
    for (int w = 1; w < 16; ++w)
      if (bv[w] > b || (bv[w] == b && bi[w] >= 0 && (id < 0 || bi[w] < id))) { b = bv[w]; id = bi[w]; }
    out[0] = id < 0 ? -1 : (cand ? cand[id] : id);
  }
}

// Start of a search segment: every key slot empty; with reset_panel also an
// empty panel and exact (FP64-derived) scores, no pending update.
__global__ void k_segment_start(DbsState* st, uint32_t* keys, int reset_panel) {
  if (threadIdx.x < 6) keys[threadIdx.x] = kNoKey;
  if (threadIdx.x == 0 && reset_panel) {
    st->m = -1;
    st->kpanel = 0;
    st->n_since = 0;
    st->exact = 1;
    st->need_refresh = 0;
    st->flips = 0;
  }
}

// Start of a search: the bookkeeping of the state reset, its objective and
// outputs (from the last re-formation of the fields) kept, the objective
// also recorded as the search's starting value.
__global__ void k_state_begin(DbsState* st, int n_sweeps, double eta) {
  if (threadIdx.x != 0) return;
  st->f_start = st->f;
  st->m = -1;
  st->done = 0;
  st->cursor_s = 0;
  st->cursor_pos = 0;
  st->n_acc = 0;
  st->sweeps = 0;
  st->converged = 0;
  st->n_sweeps = n_sweeps;
  st->attempts = 0;
  st->key = kNoKey;
  st->eta = eta;
  st->need_refresh = 0;
  st->flips = 0;
  st->kpanel = 0;   // the mixed search's panel and refresh bookkeeping
  st->n_since = 0;
  st->exact = 1;
  st->n_band = 0;
}

// ------------------------------------------------------------------ launchers
#define PNGF_NPL_SWITCH(npl, CALL) \
  switch (npl) {                   \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 4: CALL(4); break;        \
    case 8: CALL(8); break;        \
    case 16: CALL(16); break;      \
    case 32: CALL(32); break;      \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_score_rows(const ProbDev& P, int npl, const int32_t* cand, int ncand,
                             uint32_t* keyp, hipStream_t s) {
  if (ncand <= 0) return hipSuccess;
#define L_(N) hipLaunchKernelGGL(k_score_rows<N>, dim3(ncand), dim3(kRowThreads), 0, s, P, cand, ncand, keyp)
  PNGF_NPL_SWITCH(npl, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_score_tail(const ProbDev& P, uint32_t* keyp, hipStream_t s) {
  hipLaunchKernelGGL(k_score_tail, dim3((P.nd + 255) / 256), dim3(256), 0, s, P, keyp);
  return hipGetLastError();
}

hipError_t launch_refresh_tail(const ProbDev& P, const z64* god, z64 xb, uint32_t* keyp,
                               const double* df32, const double* dfb, double* out, double* bandp,
                               const int32_t* gate, hipStream_t s) {
  if (P.nfreq != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_refresh_tail, dim3(1), dim3(kTailThreads), 0, s, P, god, xb, keyp, df32,
                     dfb, out, bandp, gate);
  return hipGetLastError();
}

hipError_t launch_state_begin(DbsState* st, int n_sweeps, double eta, hipStream_t s) {
  hipLaunchKernelGGL(k_state_begin, dim3(1), dim3(64), 0, s, st, n_sweeps, eta);
  return hipGetLastError();
}

hipError_t launch_segment_start(const ProbDev& P, int reset_panel, hipStream_t s) {
  hipLaunchKernelGGL(k_segment_start, dim3(1), dim3(64), 0, s, P.st, P.keys, reset_panel);
  return hipGetLastError();
}

hipError_t launch_select_prep(const ProbDev& P, int forced, hipStream_t s) {
  hipLaunchKernelGGL(k_select_prep, dim3(1), dim3(kRowThreads), 0, s, P, forced);
  return hipGetLastError();
}

hipError_t launch_accept_rescore(const ProbDev& P, int npl, hipStream_t s) {
#define L_(N) hipLaunchKernelGGL(k_accept_rescore<N>, dim3(P.nd), dim3(kRowThreads), 0, s, P)
  PNGF_NPL_SWITCH(npl, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_accept_only(const ProbDev& P, int npl, hipStream_t s) {
#define L_(N) hipLaunchKernelGGL(k_accept_only<N>, dim3(P.nd), dim3(kRowThreads), 0, s, P)
  PNGF_NPL_SWITCH(npl, L_)
#undef L_
  return hipGetLastError();
}

// Gradient of f with respect to the relative permittivity of every pixel
// (Supplementary Note 5, eq. supp_grad_chainrule, in field form): a change d
// of eps at pixel m changes x_f by k0^2 d E_f[m] R'_f[m] to first order (R'
// is the adjoint row of the current design), and with the Wirtinger
// derivative conj(x_f) of |x_f|^2,
//     df/deps_m = sum_f coef_f 2 Re[conj(x_f) k0^2 E_f[m] R'_f[m]].
// O(N_d F) from the maintained E and R'; one thread per pixel.
__global__ __launch_bounds__(256) void k_gradient(ProbDev P, double* out) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= P.nd) return;
  double g = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    const z64 v = zmul(P.E[f][m], P.Rp[f][m]);
    const z64 x = P.st->x[f];
    g += P.coef[f] * 2.0 * P.k0sq[f] * (x.re * v.re + x.im * v.im);
  }
  out[m] = g;
}

hipError_t launch_gradient(const ProbDev& P, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gradient, dim3((P.nd + 255) / 256), dim3(256), 0, s, P, out);
  return hipGetLastError();
}

hipError_t launch_pick_best(const double* df, const int32_t* cand, int n, const DbsState* st,
                            int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pick_best, dim3(1), dim3(1024), 0, s, df, cand, n, st, out);
  return hipGetLastError();
}

}  // namespace pngf
