// One-kernel-per-step DBS kernels of libpngf (gfx950).
//
// Step t of a search is a single launch.  Every workgroup first decodes the
// pending decision from the previous step's result (the minimum visiting key,
// Results, Direct binary search: first improving flip in the visiting order)
// and forms the update scalars itself; workgroup 0 also writes the next device
// state.  Then workgroup i applies the accepted flip to row i and scores
// candidate i of the new state.  A step reads one buffer set (state, vectors,
// design bits and, on the FP64 path, C^-1) and writes the other, and the
// visiting keys rotate through three slots, so no workgroup reads anything
// another workgroup of the same launch writes.
//
// FP64 path (Sherman-Morrison, eq. lru_woodbury with M = 1):
//     C^-1_out[i,:] = C^-1_in[i,:] + alpha p_i q,  p_i = C^-1_in[i,:] . g_m,
//     q = C^-1_in[m,:],  then tau_i = C^-1_out[i,:] . G[i,:]  (3 N_d^2 x 16 B).
// Mixed path (complex-FP32 C0^-1, deferred panel):
//     p_i = C0^-1[i,:] . g_m + sum_k alpha_k p_k[m] p_k[i],
//     tau_i += alpha p_i^2   (reciprocity: (G q)_i = p_i),      (N_d^2 x 8 B)
// with p appended to the panel; E, R', tau stay FP64.
// R-form (reduced exact scoring): by reciprocity T = C^-1 G is symmetric and
// the accept of m changes it by alpha p p^T with p = T[:, m], so
//     p_i = T0[m, i] + sum_k alpha_k p_k[m] p_k[i],   tau_i += alpha p_i^2,
// with T0 = C^-1 G of the run start and the p_k kept in an FP64 panel: a
// step moves O(N_d k) bytes instead of O(N_d^2), all in FP64.
#include "dev_state.h"

namespace pngf {

__device__ __forceinline__ z64 up32(z32 a) { return {double(a.re), double(a.im)}; }

// The preloaded value for frequency 0, else a load (by value: selecting
// between a local and a global lvalue would force the local into scratch).
__device__ __forceinline__ z64 pick0(int f, z64 pre, const z64* p) {
  if (f == 0) return pre;
  return *p;
}

// Scalar view of the fields a step changes (a local copy of the whole state
// would live in scratch memory).
struct StepScalars {
  int32_t done, need_refresh, cursor_s, cursor_pos, n_acc, sweeps, converged, n_sweeps;
  int32_t n_since, kpanel, exact, flips;
  int64_t attempts;
  double f, eta;
};

// Decision context shared by a workgroup (LDS), including the changed scalars
// of the next state for the publishing workgroup.
struct StepCtx {
  int m, dpar, slot;
  int cs, cp, ns;     // cursor of the new state
  double f, eta;
  z64 alpha[kMaxFreq], Em[kMaxFreq], Rpm[kMaxFreq], x[kMaxFreq];
  StepScalars st;
};

// Decode the minimum key of the previous step into an accepted pixel and
// advance the cursor (same rules as the sequential search).  Returns m or -1
// (search ended: done/converged set).
__device__ inline int decode_key(StepScalars& st, uint32_t key, const ProbDev& P) {
  const int nd = P.nd;
  const int s = st.cursor_s, c = st.cursor_pos, ns = st.n_sweeps;
  if (key == kNoKey) {
    const bool next = (c > 0) && (s + 1 < ns);
    st.attempts += (nd - c) + (next ? nd : 0);
    st.converged = (c == 0) || next;
    st.sweeps = s + 1 + (next ? 1 : 0);
    st.done = 1;
    return -1;
  }
  int s2 = s, pos = key_vis(key);
  if (pos >= nd) {
    s2 = s + 1;
    pos -= nd;
    st.attempts += (nd - c) + pos + 1;
  } else {
    st.attempts += pos - c + 1;
  }
  const int m = key_pixel(key);
  st.sweeps = s2 + 1;
  if (pos + 1 < nd) {
    st.cursor_s = s2;
    st.cursor_pos = pos + 1;
  } else {
    st.cursor_s = s2 + 1;
    st.cursor_pos = 0;
  }
  return m;
}

__device__ __forceinline__ uint32_t step_key(const ProbDev& P, const StepCtx& c, int i) {
  if (c.cs >= c.ns) return kNoKey;
  const int pos = P.rank[size_t(c.cs) * P.nd + i];
  if (pos >= c.cp) return pack_key(pos, i);
  if (c.cs + 1 < c.ns) return pack_key(P.nd + P.rank[size_t(c.cs + 1) * P.nd + i], i);
  return kNoKey;
}

// The state scalars of a step's input state.
__device__ inline StepScalars load_scalars(const DbsState* sin) {
  StepScalars st;
  st.done = sin->done;
  st.need_refresh = sin->need_refresh;
  st.cursor_s = sin->cursor_s;
  st.cursor_pos = sin->cursor_pos;
  st.n_acc = sin->n_acc;
  st.sweeps = sin->sweeps;
  st.converged = sin->converged;
  st.n_sweeps = sin->n_sweeps;
  st.n_since = sin->n_since;
  st.kpanel = sin->kpanel;
  st.exact = sin->exact;
  st.flips = sin->flips;
  st.attempts = sin->attempts;
  st.f = sin->f;
  st.eta = sin->eta;
  return st;
}

// Loads of values that another workgroup of the same launch wrote (CO:
// device-coherent atomic loads, which bypass the non-coherent caches).
template <bool CO>
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  if constexpr (CO) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool CO>
__device__ __forceinline__ z64 ld_z64(const z64* p) {
  if constexpr (CO) {
    const uint64_t* q = reinterpret_cast<const uint64_t*>(p);
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return z64{__longlong_as_double(static_cast<long long>(a)),
               __longlong_as_double(static_cast<long long>(b))};
  } else {
    return *p;
  }
}
template <bool CO>
__device__ __forceinline__ z32 ld_z32(const z32* p) {
  if constexpr (CO) {
    const uint64_t a = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return z32{__uint_as_float(uint32_t(a)), __uint_as_float(uint32_t(a >> 32))};
  } else {
    return *p;
  }
}
template <bool CO>
__device__ __forceinline__ uint8_t ld_u8(const uint8_t* p) {
  if constexpr (CO) {
    // the aligned word holding the byte (little endian)
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const uint32_t w = __hip_atomic_load(reinterpret_cast<const uint32_t*>(a & ~uintptr_t(3)),
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return uint8_t(w >> (8 * (a & 3)));
  } else {
    return *p;
  }
}

// Stores of values that another workgroup of the same launch reads
// (device-coherent atomic stores: written through to memory).
__device__ __forceinline__ void st_z64c(z64* p, z64 v) {
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
  __hip_atomic_store(q, static_cast<uint64_t>(__double_as_longlong(v.re)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, static_cast<uint64_t>(__double_as_longlong(v.im)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_z32c(z32* p, z32 v) {
  const uint64_t a = uint64_t(__float_as_uint(v.re)) | (uint64_t(__float_as_uint(v.im)) << 32);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), a, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u8c(uint8_t* p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u32c(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: decide from the input scalars st and outputs xin, fill the
// context (c.st and c.x become the next state's).
// First half of a decision: from the step's keys, the accepted pixel (or -1
// with done / need_refresh set in st).
__device__ inline int decide_pick(const ProbDev& P, bool mixed, StepScalars& st, uint32_t key,
                                  uint32_t km) {
  int m = -1;
  if (!st.done && !st.need_refresh) {
    if (st.n_acc >= P.max_acc || st.cursor_s >= st.n_sweeps) {
      st.done = 1;
      st.converged = 0;
    } else if (mixed && !st.exact && km != kNoKey && (key == kNoKey || km < key)) {
      st.need_refresh = 2;   // a band candidate comes first: decide on FP64 state
    } else if (mixed && !st.exact &&
               ((P.k_refresh > 0 && st.n_since >= P.k_refresh) || st.kpanel >= P.kcap)) {
      st.need_refresh = 1;
    } else {
      m = decode_key(st, key, P);
    }
  }
  return m;
}

// Second half: the accepted pixel's coefficients and the new outputs; fills
// the context (c.st and c.x become the next state's).
template <bool CO>
__device__ inline void decide_apply(const ProbDev& P, int dpar, bool mixed, StepScalars st, int m,
                                    const z64* xin, StepCtx& c) {
  int slot = -1;
  if (m >= 0) {
    const uint8_t* bin = dpar ? P.bitsB : P.bits;
    const double delta = ld_u8<CO>(bin + m) ? -P.deps : P.deps;
    double fnew = 0.0;
    for (int f = 0; f < P.nfreq; ++f) {
      const double kd = P.k0sq[f] * delta;
      const z64 tau = ld_z64<CO>((dpar ? P.tauB[f] : P.tau[f]) + m);
      const z64 den = {1.0 - kd * tau.re, -kd * tau.im};
      const z64 alpha = zdiv(z64{kd, 0.0}, den);
      const z64 Em = ld_z64<CO>((dpar ? P.EB[f] : P.E[f]) + m);
      const z64 Rpm = ld_z64<CO>((dpar ? P.RpB[f] : P.Rp[f]) + m);
      c.alpha[f] = alpha;
      c.Em[f] = Em;
      c.Rpm[f] = Rpm;
      const z64 x = zfma(zmul(alpha, Em), Rpm, xin[f]);
      c.x[f] = x;
      fnew += P.coef[f] * zabs2(x);
    }
    st.f = fnew;
    st.n_acc += 1;
    st.flips += 1;
    if (mixed) {
      slot = st.kpanel;
      st.kpanel = slot + 1;
      st.n_since += 1;
      st.exact = 0;
    }
  } else {
    for (int f = 0; f < P.nfreq; ++f) c.x[f] = xin[f];
  }
  c.m = m;
  c.dpar = dpar;
  c.slot = slot;
  c.cs = st.cursor_s;
  c.cp = st.cursor_pos;
  c.ns = st.n_sweeps;
  c.f = st.f;
  c.eta = st.eta;
  c.st = st;
}

// Thread 0: decide from the input scalars st and outputs xin, fill the
// context.
__device__ inline void decide_core(const ProbDev& P, int spar, int kslot, bool mixed,
                                   StepScalars st, const z64* xin, StepCtx& c) {
  const int m = decide_pick(P, mixed, st, P.keys[kslot], P.keys[3 + kslot]);
  decide_apply<false>(P, spar, mixed, st, m, xin, c);
}

// Thread 0: read the state of this step, decide, fill the context.
__device__ inline void step_decide(const ProbDev& P, int spar, int kslot, bool mixed,
                                   StepCtx& c) {
  const DbsState* sin = spar ? P.stB : P.st;
  z64 xin[kMaxFreq];
  for (int f = 0; f < P.nfreq; ++f) xin[f] = sin->x[f];
  decide_core(P, spar, kslot, mixed, load_scalars(sin), xin, c);
}

// The publishing workgroup (all its threads, after the barrier that follows
// step_decide): the next state is the input state with this step's changes;
// the copy is spread over the workgroup, the changes written by thread 0.
// Also clears the key slot two steps ahead and logs the accept.
__device__ inline void step_publish(const ProbDev& P, int spar, int kslot, bool mixed,
                                    const StepCtx& c) {
  const DbsState* sin = spar ? P.stB : P.st;
  DbsState* sout = spar ? P.st : P.stB;
  const uint64_t* src = reinterpret_cast<const uint64_t*>(sin);
  uint64_t* dst = reinterpret_cast<uint64_t*>(sout);
  constexpr int nw = int(sizeof(DbsState) / 8);
  for (int w = threadIdx.x; w < nw; w += blockDim.x) dst[w] = src[w];
  __syncthreads();
  if (threadIdx.x == 0) {
    const StepScalars& st = c.st;
    const int m = c.m, slot = c.slot;
    sout->done = st.done;
    sout->need_refresh = st.need_refresh;
    sout->cursor_s = st.cursor_s;
    sout->cursor_pos = st.cursor_pos;
    sout->n_acc = st.n_acc;
    sout->sweeps = st.sweeps;
    sout->converged = st.converged;
    sout->n_since = st.n_since;
    sout->kpanel = st.kpanel;
    sout->exact = st.exact;
    sout->flips = st.flips;
    sout->attempts = st.attempts;
    sout->f = st.f;
    sout->m = m;
    sout->kslot = slot;
    for (int f = 0; f < P.nfreq; ++f) sout->x[f] = c.x[f];
    const int clr = (kslot + 2) % 3;
    P.keys[clr] = kNoKey;
    P.keys[3 + clr] = kNoKey;
    if (m >= 0) {
      P.log_pix[st.n_acc - 1] = m;
      P.log_f[st.n_acc - 1] = st.f;
      if (mixed) {
        P.pm[slot] = m;
        for (int f = 0; f < P.nfreq; ++f) P.alph[f][slot] = c.alpha[f];
      }
    }
  }
}

// Objective change of candidate i of the new state, its FP32 error bound.
__device__ __forceinline__ void score_terms(const ProbDev& P, const StepCtx& c, int f, z64 tau,
                                            z64 Ei, z64 Rpi, double delta, double& df,
                                            double& bnd) {
  const double kd = P.k0sq[f] * delta;
  const z64 den = {1.0 - kd * tau.re, -kd * tau.im};
  const z64 dx = zdiv(zscale(zmul(Ei, Rpi), kd), den);
  const z64 x = c.x[f];
  const double adx2 = zabs2(dx);
  df += P.coef[f] * (2.0 * (x.re * dx.re + x.im * dx.im) + adx2);
  bnd += P.coef[f] * (2.0 * sqrt(zabs2(x) * adx2) + adx2);
}

// Every step that updates reads the buffer set of its own parity (a segment
// starts at step 0 with the A set current, and each update flips the set), so
// row i of C^-1 and of G is streamed before the decision is known.
template <int NPL>
__device__ inline void plain_step_row(const ProbDev& P, int i, int spar, int kslot, StepCtx& c) {
  __shared__ double red[2 * (kRowThreads / 64)];
  const int tid = threadIdx.x;
  const int dp = spar;
  // the row of C^-1 lives in registers; G's row is read in the tau pass
  // (holding both would halve the waves per SIMD at 32 entries per lane)
  z64 row[NPL];
  if (P.nfreq == 1) {
    const z64* ci = (dp ? P.CinvB[0] : P.Cinv[0]) + size_t(i) * P.ld;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) row[t] = ci[j];
    }
  }
  // this row's vector entries, also independent of the decision
  const uint8_t* bin = dp ? P.bitsB : P.bits;
  uint8_t* bout = dp ? P.bits : P.bitsB;
  z64 e0{0.0, 0.0}, r0{0.0, 0.0};
  uint8_t b0 = 0;
  if (tid == 0) {
    b0 = bin[i];
    e0 = (dp ? P.EB[0] : P.E[0])[i];
    r0 = (dp ? P.RpB[0] : P.Rp[0])[i];
    step_decide(P, spar, kslot, false, c);
  }
  __syncthreads();
  if (i == 0) step_publish(P, spar, kslot, false, c);
  const int m = c.m;
  if (m < 0) return;
  const uint8_t bit = b0 ^ (i == m ? 1 : 0);
  const double delta = bit ? -P.deps : P.deps;
  double df = 0.0, bnd = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    const z64* Cin = (dp ? P.CinvB[f] : P.Cinv[f]);
    z64* Cout = (dp ? P.Cinv[f] : P.CinvB[f]);
    const z64* ci = Cin + size_t(i) * P.ld;
    const z64* q = Cin + size_t(m) * P.ld;
    const z64* gm = P.G[f] + size_t(m) * P.ld;
    const z64* Gi = P.G[f] + size_t(i) * P.ld;
    z64* co = Cout + size_t(i) * P.ld;
    if (f > 0 || P.nfreq != 1) {   // frequency 0 was preloaded only when alone
#pragma unroll
      for (int t = 0; t < NPL; ++t) {
        const int j = tid + t * kRowThreads;
        if (j < P.nd) row[t] = ci[j];
      }
    }
    z64 acc{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) acc = zfma(row[t], gm[j], acc);
    }
    const z64 p = block_zsum(acc, red);
    const z64 ap = zmul(c.alpha[f], p);
    acc = z64{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int j = tid + t * kRowThreads;
      if (j < P.nd) {
        row[t] = zfma(ap, q[j], row[t]);
        co[j] = row[t];
        acc = zfma(row[t], Gi[j], acc);
      }
    }
    const z64 tau = block_zsum(acc, red);
    if (tid == 0) {
      const z64 Ein = pick0(f, e0, (dp ? P.EB[f] : P.E[f]) + i);
      const z64 Rin = pick0(f, r0, (dp ? P.RpB[f] : P.Rp[f]) + i);
      const z64 Ei = zadd(Ein, zmul(ap, c.Em[f]));
      const z64 Rpi = zadd(Rin, zmul(ap, c.Rpm[f]));
      (dp ? P.E[f] : P.EB[f])[i] = Ei;
      (dp ? P.Rp[f] : P.RpB[f])[i] = Rpi;
      (dp ? P.tau[f] : P.tauB[f])[i] = tau;
      score_terms(P, c, f, tau, Ei, Rpi, delta, df, bnd);
    }
  }
  if (tid == 0) {
    bout[i] = bit;
    P.df[i] = df;
    if (df > c.eta * c.f) {
      const uint32_t k = step_key(P, c, i);
      if (k != kNoKey) atomicMin(&P.keys[(kslot + 1) % 3], k);
    }
  }
}

// Mixed step over a group of 4 RPW rows, RPW per wave: the wave streams its
// C0^-1 rows against g_m with 16-byte loads (two complex entries per lane
// and row; g_m read once for the wave's rows), then lane h < RPW forms p for
// row h, updates its FP64 E, R', tau and scores it.  A row's arithmetic does
// not depend on RPW.
// The products of the mixed search (complex FP32 with FP32 accumulation,
// FP64 vectors).  Where the step streams C0^-1 from HBM
// (many frequencies, large N_d, a batch of problems): more bytes in flight
// per wave than 8-byte loads.
constexpr int kWideRpw = 2;
constexpr int kWideRows = 4 * kWideRpw;

template <int RPW>
__device__ inline void mixed_step_wide(const ProbDev& P, int g, int spar, int kslot, StepCtx& c,
                                       z64 (*pc)[64], bool publish) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = g * (4 * RPW) + RPW * w;   // the wave's first row
  const int dp = spar;
  // the wave's FP64 vectors (E, R', tau) at every frequency, independent of
  // the decision, into LDS
  __shared__ z64 vpre[4][kMaxFreq][RPW][3];
  for (int e = lane; e < 3 * RPW * P.nfreq; e += 64) {
    const int f = e / (3 * RPW), h = (e / 3) % RPW, v = e % 3;
    const int r = r0 + h;
    if (r < P.nd) {
      const z64* src = v == 0 ? (dp ? P.EB[f] : P.E[f])
                              : (v == 1 ? (dp ? P.RpB[f] : P.Rp[f]) : (dp ? P.tauB[f] : P.tau[f]));
      vpre[w][f][h][v] = src[r];
    }
  }
  const uint8_t* bin = dp ? P.bitsB : P.bits;
  uint8_t* bout = dp ? P.bits : P.bitsB;
  const int myr = r0 + lane;                 // lane h < 4 owns row r0 + h
  const bool mine = lane < RPW && myr < P.nd;
  const uint8_t b0 = mine ? bin[myr] : 0;
  if (tid == 0) step_decide(P, spar, kslot, true, c);
  __syncthreads();
  if (publish) step_publish(P, spar, kslot, true, c);
  const int m = c.m;
  if (m < 0) return;
  const int slot = c.slot;
  // panel coefficients alpha_k p_k[m] (reciprocity: q_k . g_m = p_k[m])
  if (tid < slot)
    for (int f = 0; f < P.nfreq; ++f)
      pc[f][tid] = zmul(P.alph[f][tid], up32(P.Pp[f][size_t(tid) * P.ld + m]));
  __syncthreads();
  const uint8_t bit = b0 ^ (myr == m ? 1 : 0);
  const double dl = bit ? -P.deps : P.deps;
  double df = 0.0, bnd = 0.0;
  const int nd2 = P.nd >> 1;
  // rows past N_d (last group) read row N_d - 1 and are discarded
  size_t roff[RPW];
#pragma unroll
  for (int h = 0; h < RPW; ++h) roff[h] = size_t(min(r0 + h, P.nd - 1)) * P.ld;
  for (int f = 0; f < P.nfreq; ++f) {
    const z32* gm = P.G32[f] + size_t(m) * P.ld;
    const float4* g4 = reinterpret_cast<const float4*>(gm);
    const float4* c4[RPW];
#pragma unroll
    for (int h = 0; h < RPW; ++h) c4[h] = reinterpret_cast<const float4*>(P.C0[f] + roff[h]);
    // this group's panel entries, issued ahead of the stream
    z32 pk[RPW];
#pragma unroll
    for (int h = 0; h < RPW; ++h)
      pk[h] = lane < slot ? P.Pp[f][size_t(lane) * P.ld + min(r0 + h, P.nd - 1)] : z32{0.f, 0.f};
    float pr[RPW], pi[RPW];
#pragma unroll
    for (int h = 0; h < RPW; ++h) pr[h] = pi[h] = 0.f;
#pragma unroll 4
    for (int j = lane; j < nd2; j += 64) {
      const float4 gv = g4[j];
#pragma unroll
      for (int h = 0; h < RPW; ++h) {
        const float4 cv = c4[h][j];
        pr[h] = fmaf(cv.x, gv.x, fmaf(-cv.y, gv.y, pr[h]));
        pi[h] = fmaf(cv.x, gv.y, fmaf(cv.y, gv.x, pi[h]));
        pr[h] = fmaf(cv.z, gv.z, fmaf(-cv.w, gv.w, pr[h]));
        pi[h] = fmaf(cv.z, gv.w, fmaf(cv.w, gv.z, pi[h]));
      }
    }
    if ((P.nd & 1) && lane == 0) {   // the last entry of an odd row
      const z32 gv = gm[P.nd - 1];
#pragma unroll
      for (int h = 0; h < RPW; ++h) {
        const z32 cv = P.C0[f][roff[h] + P.nd - 1];
        pr[h] = fmaf(cv.re, gv.re, fmaf(-cv.im, gv.im, pr[h]));
        pi[h] = fmaf(cv.re, gv.im, fmaf(cv.im, gv.re, pi[h]));
      }
    }
    if (lane < slot) {
      const z64 cc = pc[f][lane];
#pragma unroll
      for (int h = 0; h < RPW; ++h) {
        pr[h] += float(cc.re * pk[h].re - cc.im * pk[h].im);
        pi[h] += float(cc.re * pk[h].im + cc.im * pk[h].re);
      }
    }
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int h = 0; h < RPW; ++h) {
      const float a = wave_sumf(pr[h]), b = wave_sumf(pi[h]);
      if (lane == h) {
        sr = a;
        si = b;
      }
    }
    if (mine) {
      const z32 p32{sr, si};
      P.Pp[f][size_t(slot) * P.ld + myr] = p32;
      const z64 p = up32(p32);
      const z64 ap = zmul(c.alpha[f], p);
      const z64 Ein = vpre[w][f][lane][0];
      const z64 Rin = vpre[w][f][lane][1];
      const z64 Tin = vpre[w][f][lane][2];
      const z64 Ei = zadd(Ein, zmul(ap, c.Em[f]));
      const z64 Rpi = zadd(Rin, zmul(ap, c.Rpm[f]));
      const z64 tau = zadd(Tin, zmul(ap, p));
      (dp ? P.E[f] : P.EB[f])[myr] = Ei;
      (dp ? P.Rp[f] : P.RpB[f])[myr] = Rpi;
      (dp ? P.tau[f] : P.tauB[f])[myr] = tau;
      score_terms(P, c, f, tau, Ei, Rpi, dl, df, bnd);
    }
  }
  if (mine) {
    bout[myr] = bit;
    P.df32[myr] = df;
    P.dfb[myr] = bnd;
    const double margin = df - c.eta * c.f;
    const double band = P.band * bnd;
    if (margin >= -band) {
      const uint32_t k = step_key(P, c, myr);
      if (k != kNoKey) atomicMin(&P.keys[(margin > band ? 0 : 3) + (kslot + 1) % 3], k);
    }
  }
}

// Single-frequency mixed step for rows of at most 64 PRE columns, with the
// decision split from the streaming: wave 0 only decides (its thread 0 issues
// no loads ahead of the state and key reads, whose wait would otherwise also
// cover every earlier load of the wave), while waves 1-4 load their two
// C0^-1 rows whole into registers meanwhile.  After the decision the g_m
// chunks are issued together, so the GEMV costs about one memory round trip.
// Same arithmetic as mixed_step_wide (FP32 products, FP64 vectors).
constexpr int kSplitThreads = 64 * (1 + kMixRows / 2);

template <int PRE>
__global__ __launch_bounds__(kSplitThreads) void k_mixed_step_split(ProbDev P, int spar,
                                                                    int kslot) {
  __shared__ StepCtx c;
  const int g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool worker = w > 0;
  const int ra = g * kMixRows + 2 * (w - 1), rb = ra + 1;
  const bool va = worker && ra < P.nd, vb = worker && rb < P.nd;
  const int dp = spar;
  z32 pa[PRE], pb[PRE];
#pragma unroll
  for (int q = 0; q < PRE; ++q) {
    const int j = lane + 64 * q;
    pa[q] = z32{0.f, 0.f};
    pb[q] = z32{0.f, 0.f};
    if (j < P.nd) {
      if (va) pa[q] = P.C0[0][size_t(ra) * P.ld + j];
      if (vb) pb[q] = P.C0[0][size_t(rb) * P.ld + j];
    }
  }
  const uint8_t* bin = dp ? P.bitsB : P.bits;
  uint8_t* bout = dp ? P.bits : P.bitsB;
  z64 e0a{0.0, 0.0}, r0a{0.0, 0.0}, t0a{0.0, 0.0}, e0b{0.0, 0.0}, r0b{0.0, 0.0}, t0b{0.0, 0.0};
  uint8_t b0a = 0, b0b = 0;
  // visiting positions of the two rows in the sweeps the new cursor can be
  // in (the decision moves it by at most two sweeps): the key of a row needs
  // its position in the cursor's sweep and, behind the cursor, in the next
  int s0 = 0, rka[4] = {0, 0, 0, 0}, rkb[4] = {0, 0, 0, 0};
  if (lane == 0 && worker) {
    const DbsState* sin = spar ? P.stB : P.st;
    s0 = sin->cursor_s;
    const int ns = sin->n_sweeps;
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (s0 + d < ns) {
        if (va) rka[d] = P.rank[size_t(s0 + d) * P.nd + ra];
        if (vb) rkb[d] = P.rank[size_t(s0 + d) * P.nd + rb];
      }
  }
  if (lane == 0 && worker) {
    if (va) {
      b0a = bin[ra];
      e0a = (dp ? P.EB[0] : P.E[0])[ra];
      r0a = (dp ? P.RpB[0] : P.Rp[0])[ra];
      t0a = (dp ? P.tauB[0] : P.tau[0])[ra];
    }
    if (vb) {
      b0b = bin[rb];
      e0b = (dp ? P.EB[0] : P.E[0])[rb];
      r0b = (dp ? P.RpB[0] : P.Rp[0])[rb];
      t0b = (dp ? P.tauB[0] : P.tau[0])[rb];
    }
  }
  if (tid == 0) step_decide(P, spar, kslot, true, c);
  __syncthreads();
  if (g == 0) step_publish(P, spar, kslot, true, c);
  const int m = c.m;
  if (m < 0 || !worker) return;
  const int slot = c.slot;
  // panel coefficient alpha_k p_k[m] of this lane's slot (reciprocity:
  // q_k . g_m = p_k[m]), loaded with the g_m chunks
  z64 cc{0.0, 0.0};
  if (lane < slot) cc = zmul(P.alph[0][lane], up32(P.Pp[0][size_t(lane) * P.ld + m]));
  const z32* gm = P.G32[0] + size_t(m) * P.ld;
  z32 gv[PRE];
#pragma unroll
  for (int q = 0; q < PRE; ++q) {
    const int j = lane + 64 * q;
    gv[q] = j < P.nd ? gm[j] : z32{0.f, 0.f};
  }
  float par = 0.f, pai = 0.f, pbr = 0.f, pbi = 0.f;
#pragma unroll
  for (int q = 0; q < PRE; ++q) {
    par = fmaf(pa[q].re, gv[q].re, fmaf(-pa[q].im, gv[q].im, par));
    pai = fmaf(pa[q].re, gv[q].im, fmaf(pa[q].im, gv[q].re, pai));
    pbr = fmaf(pb[q].re, gv[q].re, fmaf(-pb[q].im, gv[q].im, pbr));
    pbi = fmaf(pb[q].re, gv[q].im, fmaf(pb[q].im, gv[q].re, pbi));
  }
  if (lane < slot) {
    if (va) {
      const z32 pk = P.Pp[0][size_t(lane) * P.ld + ra];
      par += float(cc.re * pk.re - cc.im * pk.im);
      pai += float(cc.re * pk.im + cc.im * pk.re);
    }
    if (vb) {
      const z32 pk = P.Pp[0][size_t(lane) * P.ld + rb];
      pbr += float(cc.re * pk.re - cc.im * pk.im);
      pbi += float(cc.re * pk.im + cc.im * pk.re);
    }
  }
  par = wave_sumf(par);
  pai = wave_sumf(pai);
  pbr = wave_sumf(pbr);
  pbi = wave_sumf(pbi);
  if (lane != 0) return;
  const uint8_t bita = b0a ^ (ra == m ? 1 : 0), bitb = b0b ^ (rb == m ? 1 : 0);
  for (int h = 0; h < 2; ++h) {
    const int r = h ? rb : ra;
    if (!(h ? vb : va)) continue;
    const z32 p32{h ? pbr : par, h ? pbi : pai};
    P.Pp[0][size_t(slot) * P.ld + r] = p32;
    const z64 p = up32(p32);
    const z64 ap = zmul(c.alpha[0], p);
    const z64 Ei = zadd(h ? e0b : e0a, zmul(ap, c.Em[0]));
    const z64 Rpi = zadd(h ? r0b : r0a, zmul(ap, c.Rpm[0]));
    const z64 tau = zadd(h ? t0b : t0a, zmul(ap, p));
    (dp ? P.E[0] : P.EB[0])[r] = Ei;
    (dp ? P.Rp[0] : P.RpB[0])[r] = Rpi;
    (dp ? P.tau[0] : P.tauB[0])[r] = tau;
    const uint8_t bit = h ? bitb : bita;
    double df = 0.0, bnd = 0.0;
    score_terms(P, c, 0, tau, Ei, Rpi, bit ? -P.deps : P.deps, df, bnd);
    bout[r] = bit;
    P.df32[r] = df;
    P.dfb[r] = bnd;
    const double margin = df - c.eta * c.f;
    const double band = P.band * bnd;
    if (margin >= -band && c.cs < c.ns) {
      // step_key from the prefetched positions (c.cs - s0 is 0, 1 or 2)
      const int* rk = h ? rkb : rka;
      const int d = c.cs - s0;
      int pos = -1;
#pragma unroll
      for (int u = 0; u < 3; ++u)
        if (u == d) pos = rk[u];
      uint32_t k = kNoKey;
      if (pos >= c.cp) {
        k = pack_key(pos, r);
      } else if (c.cs + 1 < c.ns) {
        int nxt = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (u == d) nxt = rk[u + 1];
        k = pack_key(P.nd + nxt, r);
      }
      if (k != kNoKey) atomicMin(&P.keys[(margin > band ? 0 : 3) + (kslot + 1) % 3], k);
    }
  }
}

// ------------------------------------------------------- persistent mixed search
// The mixed form's steps of one batch (one frequency) in one launch of
// resident workgroups, so that the C0^-1 rows stay in registers and a step
// costs a grid barrier instead of a kernel boundary.  Each workgroup decides every step
// itself from the same keys with its own copy of the state scalars (so the
// decisions agree across workgroups), keeps the vectors and panel entries of
// its eight rows in registers, and publishes for the others only what they
// read: the accepted pixel's vectors and panel entries, and the keys.
// Workgroup 0 logs the accepts, clears the key slot two steps ahead and
// writes the state at the end, where the one-kernel-per-step search leaves
// it.  Same arithmetic as k_mixed_step_split.
constexpr int kPersistSlots = 64;     // panel slots held in LDS (>= kcap)

// Grid barrier over 64-bit words (kBarWords, one per 128-byte line; zeroed
// when the workspace is bound): workgroup g arrives on the counter of its
// partition g % 8 (on the usual round-robin dispatch, its XCD), the last of a
// partition on the global counter, and the last partition raises every
// partition's release word to the barrier's generation; each workgroup polls
// its own partition's word, so no address takes more than a partition's
// atomics or polls.  Generations keep counting across launches: the base is
// read at a launch's start and advanced by workgroup 0 at its end, so no
// launch has to clear the words.  Every wave waits for its stores and atomics
// (all cross-workgroup data goes through device-coherent stores and loads)
// before its workgroup arrives.  The wait is bounded: after spin_limit polls
// the workgroup sets *flag and reports failure, and every other workgroup
// then fails at its next barrier.
constexpr int kBarLine = 16;                       // 64-bit words per 128-byte line
constexpr int kBarParts = 8;
constexpr int kBarGen = kBarLine * (2 * kBarParts + 1);   // the generation base
constexpr int kBarWords = kBarLine * (2 * kBarParts + 2);

// Before it arrives, thread 0 publishes the workgroup's minimum keys
// (wkey[w] = {sure, band} of wave w) to ksure / kband.
__device__ inline bool grid_barrier(uint64_t* bar, uint64_t gen, int spin_limit, int32_t* flag,
                                    int* ok, uint32_t* ksure, uint32_t* kband,
                                    const uint32_t (*wkey)[2]) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = kNoKey, b = kNoKey;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) {
      a = min(a, wkey[w][0]);
      b = min(b, wkey[w][1]);
    }
    if (a != kNoKey) atomicMin(ksure, a);
    if (b != kNoKey) atomicMin(kband, b);
    __builtin_amdgcn_s_waitcnt(0);
    const uint64_t G = gridDim.x, x = blockIdx.x % kBarParts;
    const uint64_t nparts = G < uint64_t(kBarParts) ? G : uint64_t(kBarParts);
    const uint64_t nx = (G - x + kBarParts - 1) / kBarParts;
    uint64_t* sub = bar + kBarLine * x;
    uint64_t* glob = bar + kBarLine * kBarParts;
    uint64_t* rel = bar + kBarLine * (kBarParts + 1);
    if (atomicAdd(reinterpret_cast<unsigned long long*>(sub), 1ull) + 1ull == gen * nx)
      if (atomicAdd(reinterpret_cast<unsigned long long*>(glob), 1ull) + 1ull == gen * nparts)
        for (uint64_t y = 0; y < nparts; ++y)
          __hip_atomic_store(rel + kBarLine * y, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int n = 0;
    bool good = true;
    while (__hip_atomic_load(rel + kBarLine * x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           gen) {
      if (++n > spin_limit) {
        good = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!good) atomicOr(flag, 1);
    *ok = good ? 1 : 0;
  }
  __syncthreads();
  return *ok != 0;
}

// Four waves of two rows each, one wave per SIMD, so a wave may hold up to
// 512 registers (its rows, the g_m chunk and the rows' state).  Wave 0 also
// decides: thread 0 picks the accepted pixel m from the keys, then thread 0
// fetches m's vectors while lane k < slot fetches the panel entry p_k[m]
// (the coefficient c_k = alpha_k p_k[m] every worker needs, into LDS).  In
// each worker, lane l < 2 holds the FP64 state of row 2w + l and updates it.
constexpr int kPersistThreads = 64 * (kMixRows / 2);

template <int PRE>
__global__ __launch_bounds__(kPersistThreads, 1) void k_mixed_persist(ProbDev P, int t0,
                                                                     int nsteps, uint64_t* bar,
                                                                     int32_t* flag,
                                                                     int spin_limit,
                                                                     const double* bandp,
                                                                     const int32_t* wstat) {
  __shared__ StepCtx c;
  __shared__ z64 alph_s[kPersistSlots];
  __shared__ z64 cc_s[kPersistSlots];
  __shared__ StepScalars s_st;
  __shared__ int s_m;
  __shared__ int s_ok;
  __shared__ uint64_t s_gen;
  __shared__ uint32_t wkey_s[kPersistThreads / 64][2];
  const int g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ra = g * kMixRows + 2 * w, rb = ra + 1;
  const bool va = ra < P.nd, vb = rb < P.nd;
  const int rown = ra + (lane & 1);           // the row of lane 0 / 1
  const bool vown = lane < 2 && rown < P.nd;
  // acquire: nothing of the previous launches' writes may be read stale
  if (tid == 0) __threadfence();
  __syncthreads();
  // a block-Woodbury refresh enqueued before this launch that found its
  // capacitance matrix singular: C0^-1 is unusable, so no step runs (every
  // workgroup reads the same word); the host re-inverts and launches again
  if (wstat && *wstat) {
    if (g == 0 && tid == 0) *flag = 2;
    return;
  }
  const double bandv = *bandp;   // the error band, set on the device by the last refresh
  z32 pa[PRE], pb[PRE];
#pragma unroll
  for (int q = 0; q < PRE; ++q) {
    const int j = lane + 64 * q;
    pa[q] = z32{0.f, 0.f};
    pb[q] = z32{0.f, 0.f};
    if (j < P.nd) {
      if (va) pa[q] = P.C0[0][size_t(ra) * P.ld + j];
      if (vb) pb[q] = P.C0[0][size_t(rb) * P.ld + j];
    }
  }
  // the own row's vectors as of the batch start
  const int sp0 = t0 & 1;
  z64 e{0.0, 0.0}, rp{0.0, 0.0}, ta{0.0, 0.0};
  uint8_t bit = 0;
  if (vown) {
    bit = (sp0 ? P.bitsB : P.bits)[rown];
    e = (sp0 ? P.EB[0] : P.E[0])[rown];
    rp = (sp0 ? P.RpB[0] : P.Rp[0])[rown];
    ta = (sp0 ? P.tauB[0] : P.tau[0])[rown];
  }
  if (tid == 0) {
    const DbsState* sin = sp0 ? P.stB : P.st;
    c.st = load_scalars(sin);
    c.x[0] = sin->x[0];
    s_gen = bar[kBarGen];
  }
  for (int i = tid; i < kPersistSlots; i += blockDim.x) alph_s[i] = P.alph[0][i];
  __syncthreads();
  // panel entries p_k[r] of the two rows for the slots filled before the batch
  const int k_start = c.st.kpanel;
  z32 ppa{0.f, 0.f}, ppb{0.f, 0.f};
  if (lane < k_start) {
    if (va) ppa = P.Pp[0][size_t(lane) * P.ld + ra];
    if (vb) ppb = P.Pp[0][size_t(lane) * P.ld + rb];
  }
  int it = 0;
  bool alive = true;
  for (; it < nsteps; ++it) {
    const int t = t0 + it, dp = t & 1, kslot = t % 3;
    // pick the accepted pixel first: the g_m loads and products of every
    // wave then overlap the second half of the decision
    if (tid == 0) {
      StepScalars st = c.st;
      s_m = decide_pick(P, true, st, ld_u32<true>(P.keys + kslot),
                        ld_u32<true>(P.keys + 3 + kslot));
      s_st = st;
    }
    __syncthreads();
    const int m = s_m;
    if (m < 0) {
      if (tid == 0) {
        const z64 xin = c.x[0];
        decide_apply<true>(P, dp, true, s_st, -1, &xin, c);
        if (g == 0) {
          const int clr = (kslot + 2) % 3;
          st_u32c(P.keys + clr, kNoKey);
          st_u32c(P.keys + 3 + clr, kNoKey);
        }
      }
      break;
    }
    const z32* gm = P.G32[0] + size_t(m) * P.ld;
    z32 gv[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int j = lane + 64 * q;
      gv[q] = j < P.nd ? gm[j] : z32{0.f, 0.f};
    }
    if (w == 0) {
      if (lane < s_st.kpanel)
        cc_s[lane] = zmul(alph_s[lane], up32(ld_z32<true>(P.Pp[0] + size_t(lane) * P.ld + m)));
      if (lane == 0) {
        const z64 xin = c.x[0];
        decide_apply<true>(P, dp, true, s_st, m, &xin, c);
        alph_s[c.slot] = c.alpha[0];
      }
    }
    float par = 0.f, pai = 0.f, pbr = 0.f, pbi = 0.f;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      par = fmaf(pa[q].re, gv[q].re, fmaf(-pa[q].im, gv[q].im, par));
      pai = fmaf(pa[q].re, gv[q].im, fmaf(pa[q].im, gv[q].re, pai));
      pbr = fmaf(pb[q].re, gv[q].re, fmaf(-pb[q].im, gv[q].im, pbr));
      pbi = fmaf(pb[q].re, gv[q].im, fmaf(pb[q].im, gv[q].re, pbi));
    }
    __syncthreads();
    if (g == 0 && tid == 0) {
      const int clr = (kslot + 2) % 3;
      st_u32c(P.keys + clr, kNoKey);
      st_u32c(P.keys + 3 + clr, kNoKey);
      P.log_pix[c.st.n_acc - 1] = m;
      P.log_f[c.st.n_acc - 1] = c.st.f;
      P.pm[c.slot] = m;
      P.alph[0][c.slot] = c.alpha[0];
    }
    const int slot = c.slot;
    uint32_t ksure = kNoKey, kband = kNoKey;
    {
      // visiting positions of the own row in the new cursor's sweep and the next
      int pk = -1, nk = 0;
      if (vown && c.cs < c.ns) {
        pk = P.rank[size_t(c.cs) * P.nd + rown];
        if (c.cs + 1 < c.ns) nk = P.rank[size_t(c.cs + 1) * P.nd + rown];
      }
      if (lane < slot) {
        const z64 cc = cc_s[lane];
        if (va) {
          par += float(cc.re * ppa.re - cc.im * ppa.im);
          pai += float(cc.re * ppa.im + cc.im * ppa.re);
        }
        if (vb) {
          pbr += float(cc.re * ppb.re - cc.im * ppb.im);
          pbi += float(cc.re * ppb.im + cc.im * ppb.re);
        }
      }
      par = wave_sumf(par);
      pai = wave_sumf(pai);
      pbr = wave_sumf(pbr);
      pbi = wave_sumf(pbi);
      if (lane == slot) {
        ppa = z32{par, pai};
        ppb = z32{pbr, pbi};
      }
      if (vown) {
        const int r = rown;
        const z32 p32 = (lane & 1) ? z32{pbr, pbi} : z32{par, pai};
        st_z32c(P.Pp[0] + size_t(slot) * P.ld + r, p32);
        const z64 p = up32(p32);
        const z64 ap = zmul(c.alpha[0], p);
        e = zadd(e, zmul(ap, c.Em[0]));
        rp = zadd(rp, zmul(ap, c.Rpm[0]));
        ta = zadd(ta, zmul(ap, p));
        bit = bit ^ (r == m ? 1 : 0);
        st_z64c((dp ? P.E[0] : P.EB[0]) + r, e);
        st_z64c((dp ? P.Rp[0] : P.RpB[0]) + r, rp);
        st_z64c((dp ? P.tau[0] : P.tauB[0]) + r, ta);
        double df = 0.0, bnd = 0.0;
        score_terms(P, c, 0, ta, e, rp, bit ? -P.deps : P.deps, df, bnd);
        st_u8c((dp ? P.bits : P.bitsB) + r, bit);
        P.df32[r] = df;
        P.dfb[r] = bnd;
        const double margin = df - c.eta * c.f;
        const double band = bandv * bnd;
        if (margin >= -band && c.cs < c.ns) {
          uint32_t k = kNoKey;
          if (pk >= c.cp) k = pack_key(pk, r);
          else if (c.cs + 1 < c.ns) k = pack_key(P.nd + nk, r);
          if (margin > band) ksure = k;
          else kband = k;
        }
      }
    }
    // the workgroup's minimum keys (sure, band): one atomic each per
    // workgroup instead of one per row
    ksure = min(ksure, uint32_t(__shfl_xor(int(ksure), 1, 64)));
    kband = min(kband, uint32_t(__shfl_xor(int(kband), 1, 64)));
    if (lane == 0) {
      wkey_s[w][0] = ksure;
      wkey_s[w][1] = kband;
    }
    if (!grid_barrier(bar, s_gen + uint64_t(it + 1), spin_limit, flag, &s_ok,
                      P.keys + (kslot + 1) % 3, P.keys + 3 + (kslot + 1) % 3, wkey_s)) {
      alive = false;
      break;
    }
  }
  if (g == 0 && tid == 0 && alive) {
    // every workgroup met the same `it` barriers
    bar[kBarGen] = s_gen + uint64_t(it);
    // the state where the last of nsteps one-step launches writes it
    const DbsState* sin = sp0 ? P.stB : P.st;
    DbsState* sout = ((t0 + nsteps - 1) & 1) ? P.st : P.stB;
    if (sout != sin) {
      const uint64_t* src = reinterpret_cast<const uint64_t*>(sin);
      uint64_t* dst = reinterpret_cast<uint64_t*>(sout);
      for (int i = 0; i < int(sizeof(DbsState) / 8); ++i) dst[i] = src[i];
    }
    const StepScalars& st = c.st;
    sout->done = st.done;
    sout->need_refresh = st.need_refresh;
    sout->cursor_s = st.cursor_s;
    sout->cursor_pos = st.cursor_pos;
    sout->n_acc = st.n_acc;
    sout->sweeps = st.sweeps;
    sout->converged = st.converged;
    sout->n_since = st.n_since;
    sout->kpanel = st.kpanel;
    sout->exact = st.exact;
    sout->flips = st.flips;
    sout->attempts = st.attempts;
    sout->f = st.f;
    sout->m = c.m;
    sout->kslot = c.slot;
    sout->x[0] = c.x[0];
  }
  // release: every write of this launch reaches memory before it ends
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) __threadfence();
}

// Several-frequency mixed step for rows of at most 64 PRE columns: one
// workgroup per row pair, wave 0 decides, worker wave 1 + f handles frequency
// f of both rows (its C0^-1 rows of that frequency are loaded whole during the
// decision), and the frequencies' score terms meet in LDS, where wave 1 sums
// them and publishes the keys.  Same arithmetic as mixed_step_wide.
constexpr int kMfMaxThreads = 64 * (1 + kMaxFreq);

template <int PRE>
__global__ __launch_bounds__(kMfMaxThreads) void k_mixed_step_mf(ProbDev P, int spar, int kslot) {
  __shared__ StepCtx c;
  __shared__ double sdf[kMaxFreq][2], sbnd[kMaxFreq][2];
  const int g = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int f = w - 1;                       // frequency of a worker wave
  const bool worker = w > 0 && f < P.nfreq;
  const int ra = 2 * g, rb = ra + 1;
  const bool va = worker && ra < P.nd, vb = worker && rb < P.nd;
  const int dp = spar;
  const int fw = worker ? f : 0;
  z32 pa[PRE], pb[PRE];
#pragma unroll
  for (int q = 0; q < PRE; ++q) {
    const int j = lane + 64 * q;
    pa[q] = z32{0.f, 0.f};
    pb[q] = z32{0.f, 0.f};
    if (j < P.nd) {
      if (va) pa[q] = P.C0[fw][size_t(ra) * P.ld + j];
      if (vb) pb[q] = P.C0[fw][size_t(rb) * P.ld + j];
    }
  }
  const uint8_t* bin = dp ? P.bitsB : P.bits;
  uint8_t* bout = dp ? P.bits : P.bitsB;
  z64 ea{0.0, 0.0}, rpa{0.0, 0.0}, ta{0.0, 0.0}, eb{0.0, 0.0}, rpb{0.0, 0.0}, tb{0.0, 0.0};
  uint8_t b0a = 0, b0b = 0;
  int s0 = 0, rka[4] = {0, 0, 0, 0}, rkb[4] = {0, 0, 0, 0};
  if (lane == 0 && worker) {
    if (va) {
      b0a = bin[ra];
      ea = (dp ? P.EB[fw] : P.E[fw])[ra];
      rpa = (dp ? P.RpB[fw] : P.Rp[fw])[ra];
      ta = (dp ? P.tauB[fw] : P.tau[fw])[ra];
    }
    if (vb) {
      b0b = bin[rb];
      eb = (dp ? P.EB[fw] : P.E[fw])[rb];
      rpb = (dp ? P.RpB[fw] : P.Rp[fw])[rb];
      tb = (dp ? P.tauB[fw] : P.tau[fw])[rb];
    }
    if (f == 0) {
      // visiting positions for the keys (see k_mixed_step_split)
      const DbsState* sin = spar ? P.stB : P.st;
      s0 = sin->cursor_s;
      const int ns = sin->n_sweeps;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (s0 + d < ns) {
          if (va) rka[d] = P.rank[size_t(s0 + d) * P.nd + ra];
          if (vb) rkb[d] = P.rank[size_t(s0 + d) * P.nd + rb];
        }
    }
  }
  if (tid == 0) step_decide(P, spar, kslot, true, c);
  __syncthreads();
  if (g == 0) step_publish(P, spar, kslot, true, c);
  const int m = c.m;
  if (m < 0) return;
  const int slot = c.slot;
  if (worker) {
    z64 cc{0.0, 0.0};
    if (lane < slot) cc = zmul(P.alph[f][lane], up32(P.Pp[f][size_t(lane) * P.ld + m]));
    const z32* gm = P.G32[f] + size_t(m) * P.ld;
    z32 gv[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int j = lane + 64 * q;
      gv[q] = j < P.nd ? gm[j] : z32{0.f, 0.f};
    }
    float par = 0.f, pai = 0.f, pbr = 0.f, pbi = 0.f;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      par = fmaf(pa[q].re, gv[q].re, fmaf(-pa[q].im, gv[q].im, par));
      pai = fmaf(pa[q].re, gv[q].im, fmaf(pa[q].im, gv[q].re, pai));
      pbr = fmaf(pb[q].re, gv[q].re, fmaf(-pb[q].im, gv[q].im, pbr));
      pbi = fmaf(pb[q].re, gv[q].im, fmaf(pb[q].im, gv[q].re, pbi));
    }
    if (lane < slot) {
      if (va) {
        const z32 pk = P.Pp[f][size_t(lane) * P.ld + ra];
        par += float(cc.re * pk.re - cc.im * pk.im);
        pai += float(cc.re * pk.im + cc.im * pk.re);
      }
      if (vb) {
        const z32 pk = P.Pp[f][size_t(lane) * P.ld + rb];
        pbr += float(cc.re * pk.re - cc.im * pk.im);
        pbi += float(cc.re * pk.im + cc.im * pk.re);
      }
    }
    par = wave_sumf(par);
    pai = wave_sumf(pai);
    pbr = wave_sumf(pbr);
    pbi = wave_sumf(pbi);
    if (lane == 0) {
      const uint8_t bita = b0a ^ (ra == m ? 1 : 0), bitb = b0b ^ (rb == m ? 1 : 0);
      for (int h = 0; h < 2; ++h) {
        double df = 0.0, bnd = 0.0;
        const int r = h ? rb : ra;
        if (h ? vb : va) {
          const z32 p32{h ? pbr : par, h ? pbi : pai};
          P.Pp[f][size_t(slot) * P.ld + r] = p32;
          const z64 p = up32(p32);
          const z64 ap = zmul(c.alpha[f], p);
          const z64 Ei = zadd(h ? eb : ea, zmul(ap, c.Em[f]));
          const z64 Rpi = zadd(h ? rpb : rpa, zmul(ap, c.Rpm[f]));
          const z64 tau = zadd(h ? tb : ta, zmul(ap, p));
          (dp ? P.E[f] : P.EB[f])[r] = Ei;
          (dp ? P.Rp[f] : P.RpB[f])[r] = Rpi;
          (dp ? P.tau[f] : P.tauB[f])[r] = tau;
          const uint8_t bit = h ? bitb : bita;
          score_terms(P, c, f, tau, Ei, Rpi, bit ? -P.deps : P.deps, df, bnd);
          if (f == 0) bout[r] = bit;
        }
        sdf[f][h] = df;
        sbnd[f][h] = bnd;
      }
    }
  }
  __syncthreads();
  if (w != 1 || lane != 0) return;
  for (int h = 0; h < 2; ++h) {
    const int r = h ? rb : ra;
    if (!(h ? vb : va)) continue;
    double df = 0.0, bnd = 0.0;
    for (int ff = 0; ff < P.nfreq; ++ff) {
      df += sdf[ff][h];
      bnd += sbnd[ff][h];
    }
    P.df32[r] = df;
    P.dfb[r] = bnd;
    const double margin = df - c.eta * c.f;
    const double band = P.band * bnd;
    if (margin >= -band && c.cs < c.ns) {
      const int* rk = h ? rkb : rka;
      const int d = c.cs - s0;
      int pos = -1;
#pragma unroll
      for (int u = 0; u < 3; ++u)
        if (u == d) pos = rk[u];
      uint32_t k = kNoKey;
      if (pos >= c.cp) {
        k = pack_key(pos, r);
      } else if (c.cs + 1 < c.ns) {
        int nxt = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (u == d) nxt = rk[u + 1];
        k = pack_key(P.nd + nxt, r);
      }
      if (k != kNoKey) atomicMin(&P.keys[(margin > band ? 0 : 3) + (kslot + 1) % 3], k);
    }
  }
}

template <int NPL>
__global__ __launch_bounds__(kRowThreads) void k_plain_step(ProbDev P, int spar, int kslot) {
  __shared__ StepCtx c;
  plain_step_row<NPL>(P, blockIdx.x, spar, kslot, c);
}

__global__ __launch_bounds__(256) void k_mixed_step(ProbDev P, int spar, int kslot) {
  __shared__ StepCtx c;
  __shared__ z64 pc[kMaxFreq][64];
  mixed_step_wide<kWideRpw>(P, blockIdx.x, spar, kslot, c, pc, blockIdx.x == 0);
}

// Batched step: one launch advances every active problem of a batch by one
// step.  Work item b (a row of one problem on the FP64 path, a group of
// 4 RPW rows on the mixed path, RPW a tuned launch shape) maps to problem p
// with row0[p] <= b <
// row0[p+1], p < *nact (the active count lives on the device, so that one
// captured launch serves any active set); the grid is either one workgroup
// per item of the whole batch (surplus workgroups exit) or a persistent grid
// that strides over the items (launch shape chosen by the autotuner).  Problems
// are independent (Results, Computational efficiency: per-frequency and
// per-design systems need no communication).
template <int NPL, bool MIXED, int RPW = kWideRpw>
__global__ __launch_bounds__(kRowThreads) void k_batch_step(const ProbDev* probs,
                                                            const int32_t* row0,
                                                            const int32_t* nact, int spar,
                                                            int kslot) {
  __shared__ StepCtx c;
  __shared__ z64 pc[kMaxFreq][64];
  const int nprob = *nact;          // problems stepped by this launch (descriptors 0..nprob-1)
  const int total = row0[nprob];
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    int lo = 0, hi = nprob - 1;       // largest p with row0[p] <= b
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (row0[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const ProbDev& P = probs[lo];
    const int i = b - row0[lo];
    __syncthreads();   // the previous item is done with the shared context
    if (MIXED) mixed_step_wide<RPW>(P, i, spar, kslot, c, pc, i == 0);
    else plain_step_row<NPL>(P, i, spar, kslot, c);
  }
}

// Panel q vectors rebuilt for a fold: q_k = C0^-1[m_k,:] + sum_{l<k} alpha_l
// p_l[m_k] q_l (the row m_k of the inverse in force when slot k was made).
// The coefficients alpha_l p_l[m_k] are formed once per workgroup in LDS.
__global__ __launch_bounds__(256) void k_fold_q(ProbDev P, int f, int kp) {
  __shared__ z64 cf[64][65];
  __shared__ int mk[64];
  const z32* Pp = P.Pp[f];
  z32* Qp = P.Qp[f];
  for (int e = threadIdx.x; e < kp * kp; e += 256) {
    const int k = e / kp, l = e % kp;
    cf[k][l] = (l < k) ? zmul(P.alph[f][l], up32(Pp[size_t(l) * P.ld + P.pm[k]])) : z64{0.0, 0.0};
  }
  if (threadIdx.x < kp) mk[threadIdx.x] = P.pm[threadIdx.x];
  __syncthreads();
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= P.nd) return;
  for (int k = 0; k < kp; ++k) {
    z64 acc = up32(P.C0[f][size_t(mk[k]) * P.ld + j]);
    for (int l = 0; l < k; ++l) acc = zfma(cf[k][l], up32(Qp[size_t(l) * P.ld + j]), acc);
    Qp[size_t(k) * P.ld + j] = z32{float(acc.re), float(acc.im)};
  }
}

// R-form step: 64 rows per workgroup, one row per lane; the four waves split
// the panel sum over slots (fixed combination order).
constexpr int kRRows = 64;
constexpr int kRCoef = 256;   // panel coefficients staged in LDS at a time

__global__ __launch_bounds__(256) void k_rform_step(ProbDev P, int spar, int kslot) {
  __shared__ StepCtx c;
  __shared__ z64 cf[kRCoef];
  __shared__ z64 part[4][kRRows];
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  const int i = blockIdx.x * kRRows + lane;
  const bool own = (q == 0) && (i < P.nd);
  const int dp = spar;
  // this row's vectors do not depend on the decision
  z64 e0{0.0, 0.0}, r0{0.0, 0.0}, t0{0.0, 0.0};
  uint8_t b0 = 0;
  if (own) {
    b0 = (dp ? P.bitsB : P.bits)[i];
    e0 = (dp ? P.EB[0] : P.E[0])[i];
    r0 = (dp ? P.RpB[0] : P.Rp[0])[i];
    t0 = (dp ? P.tauB[0] : P.tau[0])[i];
  }
  if (tid == 0) step_decide(P, spar, kslot, true, c);
  __syncthreads();
  if (blockIdx.x == 0) step_publish(P, spar, kslot, true, c);
  const int m = c.m;
  if (m < 0) return;
  const int slot = c.slot;
  const uint8_t bit = b0 ^ (i == m ? 1 : 0);
  const double delta = bit ? -P.deps : P.deps;
  double df = 0.0, bnd = 0.0;
  for (int f = 0; f < P.nfreq; ++f) {
    const z64* U = P.Up[f];
    // T0[m, i] is issued before the panel terms so the loads overlap
    z64 tmi{0.0, 0.0};
    if (own) tmi = P.T0[f][size_t(m) * P.ld + i];
    z64 acc{0.0, 0.0};
    for (int j0 = 0; j0 < slot; j0 += kRCoef) {
      const int nj = min(kRCoef, slot - j0);
      __syncthreads();   // the previous chunk of coefficients is consumed
      for (int j = tid; j < nj; j += 256)
        cf[j] = zmul(P.alph[f][j0 + j], U[size_t(j0 + j) * P.ld + m]);
      __syncthreads();
      if (i < P.nd) {
        // four independent partial sums keep several panel loads in flight
        z64 a1{0.0, 0.0}, a2{0.0, 0.0}, a3{0.0, 0.0};
        int j = q;
        for (; j + 12 < nj; j += 16) {
          acc = zfma(cf[j], U[size_t(j0 + j) * P.ld + i], acc);
          a1 = zfma(cf[j + 4], U[size_t(j0 + j + 4) * P.ld + i], a1);
          a2 = zfma(cf[j + 8], U[size_t(j0 + j + 8) * P.ld + i], a2);
          a3 = zfma(cf[j + 12], U[size_t(j0 + j + 12) * P.ld + i], a3);
        }
        for (; j < nj; j += 4) acc = zfma(cf[j], U[size_t(j0 + j) * P.ld + i], acc);
        acc = zadd(zadd(acc, a1), zadd(a2, a3));
      }
    }
    part[q][lane] = acc;
    __syncthreads();
    if (own) {
      const z64 s01 = zadd(part[0][lane], part[1][lane]);
      const z64 s23 = zadd(part[2][lane], part[3][lane]);
      const z64 p = zadd(tmi, zadd(s01, s23));
      P.Up[f][size_t(slot) * P.ld + i] = p;
      const z64 ap = zmul(c.alpha[f], p);
      const z64 Ein = pick0(f, e0, (dp ? P.EB[f] : P.E[f]) + i);
      const z64 Rin = pick0(f, r0, (dp ? P.RpB[f] : P.Rp[f]) + i);
      const z64 Tin = pick0(f, t0, (dp ? P.tauB[f] : P.tau[f]) + i);
      const z64 Ei = zadd(Ein, zmul(ap, c.Em[f]));
      const z64 Rpi = zadd(Rin, zmul(ap, c.Rpm[f]));
      const z64 tau = zadd(Tin, zmul(ap, p));
      (dp ? P.E[f] : P.EB[f])[i] = Ei;
      (dp ? P.Rp[f] : P.RpB[f])[i] = Rpi;
      (dp ? P.tau[f] : P.tauB[f])[i] = tau;
      score_terms(P, c, f, tau, Ei, Rpi, delta, df, bnd);
    }
    __syncthreads();   // part is reused by the next frequency
  }
  if (own) {
    (dp ? P.bits : P.bitsB)[i] = bit;
    P.df[i] = df;
    if (df > c.eta * c.f) {
      const uint32_t k = step_key(P, c, i);
      if (k != kNoKey) atomicMin(&P.keys[(kslot + 1) % 3], k);
    }
  }
}

// Scores of every candidate from the maintained tau, E, R' (current A set)
// into key slot 0: the start of a segment after the panel was folded.
__global__ __launch_bounds__(256) void k_rform_score(ProbDev P) {
  __shared__ StepCtx c;
  if (threadIdx.x == 0) {
    const DbsState* s = P.st;
    c.cs = s->cursor_s;
    c.cp = s->cursor_pos;
    c.ns = s->n_sweeps;
    c.f = s->f;
    c.eta = s->eta;
    for (int f = 0; f < P.nfreq; ++f) c.x[f] = s->x[f];
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= P.nd) return;
  const double delta = P.bits[i] ? -P.deps : P.deps;
  double df = 0.0, bnd = 0.0;
  for (int f = 0; f < P.nfreq; ++f)
    score_terms(P, c, f, P.tau[f][i], P.E[f][i], P.Rp[f][i], delta, df, bnd);
  P.df[i] = df;
  if (df > c.eta * c.f) {
    const uint32_t k = step_key(P, c, i);
    if (k != kNoKey) atomicMin(&P.keys[0], k);
  }
}

// Ut[i][k] = alpha_k p_k[i] (N_d x kp), the left factor of the panel fold
// T0 += Ut U.
__global__ __launch_bounds__(256) void k_rform_ut(ProbDev P, int f, int kp, z64* Ut) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= size_t(P.nd) * kp) return;
  const int i = int(e / kp), k = int(e % kp);
  Ut[e] = zmul(P.alph[f][k], P.Up[f][size_t(k) * P.ld + i]);
}

// T0 rows: G[i,:] for pixels at eps_lo, zero for pixels at eps_hi (the
// identity columns of C^-1 contribute G[Z,:]; the GEMM adds C^-1[:,S] G[S,:]).
__global__ __launch_bounds__(256) void k_rform_t0_init(ProbDev P, int f) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= P.nd) return;
  P.T0[f][size_t(i) * P.ld + j] = P.bits[i] ? z64{0.0, 0.0} : P.G[f][size_t(i) * P.ld + j];
}

// ------------------------------------------------------------------ launchers
#define PNGF_STEP_SWITCH(KERNEL, npl, ...)                                                      \
  switch (npl) {                                                                               \
    case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                                  \
    case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                                  \
    case 4: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                                  \
    case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                                  \
    case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                                \
    case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                                \
    default: return hipErrorInvalidValue;                                                      \
  }

hipError_t launch_plain_step(const ProbDev& P, int npl, int step, hipStream_t s) {
  PNGF_STEP_SWITCH(k_plain_step, npl, dim3(P.nd), dim3(kRowThreads), 0, s, P, step & 1, step % 3)
  return hipGetLastError();
}

hipError_t launch_mixed_step(const ProbDev& P, int npl, int step, hipStream_t s) {
  (void)npl;
  const dim3 grid((P.nd + kMixRows - 1) / kMixRows);
  const int sp = step & 1, ks = step % 3;
  if (P.nfreq == 1 && P.nd <= 64 * 8)
    hipLaunchKernelGGL(k_mixed_step_split<8>, grid, dim3(kSplitThreads), 0, s, P, sp, ks);
  else if (P.nfreq == 1 && P.nd <= 64 * 16)
    hipLaunchKernelGGL(k_mixed_step_split<16>, grid, dim3(kSplitThreads), 0, s, P, sp, ks);
  else if (P.nfreq == 1 && P.nd <= 64 * 32)
    hipLaunchKernelGGL(k_mixed_step_split<32>, grid, dim3(kSplitThreads), 0, s, P, sp, ks);
  else if (P.nfreq > 1 && P.nd <= 64 * 8)
    hipLaunchKernelGGL(k_mixed_step_mf<8>, dim3((P.nd + 1) / 2), dim3(64 * (1 + P.nfreq)), 0, s,
                       P, sp, ks);
  else if (P.nfreq > 1 && P.nd <= 64 * 16)
    hipLaunchKernelGGL(k_mixed_step_mf<16>, dim3((P.nd + 1) / 2), dim3(64 * (1 + P.nfreq)), 0, s,
                       P, sp, ks);
  else
    hipLaunchKernelGGL(k_mixed_step, dim3((P.nd + kWideRows - 1) / kWideRows), dim3(256), 0, s,
                       P, sp, ks);
  return hipGetLastError();
}

// The batch [t0, t0 + nsteps) of the mixed search in one launch (one
// frequency, N_d <= 2048, kcap <= kPersistSlots) whose workgroups must all be
// resident at once: hipErrorNotSupported when the form does not apply or the
// grid exceeds one wave of workgroups on this device (the grid barriers would
// then wait on workgroups not yet started; their waits are bounded in any
// case, for devices shared with other work).  bar (kBarWords 64-bit words)
// and flag are zeroed when the workspace is bound; a launch that timed out
// leaves them to be cleared by the caller.
template <int PRE>
hipError_t launch_persist_pre(const ProbDev& P, int t0, int nsteps, uint64_t* bar, int32_t* flag,
                              int spin_limit, const double* bandp, const int32_t* wstat,
                              hipStream_t s) {
  static int cap[64] = {0};       // resident workgroups per device (0: not known yet)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorNotSupported;
  if (cap[dev] == 0) {
    int per_cu = 0, ncu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mixed_persist<PRE>,
                                                     kPersistThreads, 0);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    cap[dev] = per_cu * ncu > 0 ? per_cu * ncu : -1;
  }
  const int grid = (P.nd + kMixRows - 1) / kMixRows;
  if (grid > cap[dev]) return hipErrorNotSupported;
  hipLaunchKernelGGL(k_mixed_persist<PRE>, dim3(grid), dim3(kPersistThreads), 0, s, P, t0, nsteps,
                     bar, flag, spin_limit, bandp, wstat);
  return hipGetLastError();
}

// bandp: the device word holding the error band; wstat (nullable): the
// status of a block-Woodbury refresh still unread by the host.
hipError_t launch_mixed_persist(const ProbDev& P, int t0, int nsteps, uint64_t* bar,
                                int32_t* flag, int spin_limit, const double* bandp,
                                const int32_t* wstat, hipStream_t s) {
  if (P.nfreq != 1 || P.nd > 64 * 32 || P.kcap > kPersistSlots) return hipErrorNotSupported;
  if (P.nd <= 64 * 8)
    return launch_persist_pre<8>(P, t0, nsteps, bar, flag, spin_limit, bandp, wstat, s);
  if (P.nd <= 64 * 16)
    return launch_persist_pre<16>(P, t0, nsteps, bar, flag, spin_limit, bandp, wstat, s);
  return launch_persist_pre<32>(P, t0, nsteps, bar, flag, spin_limit, bandp, wstat, s);
}

hipError_t launch_batch_step(const ProbDev* probs, const int32_t* row0, const int32_t* nact,
                             int total, int grid, int npl, int mixed, int rpw, int step,
                             hipStream_t s) {
  const int g = (grid > 0 && grid < total) ? grid : total;
  if (g <= 0) return hipSuccess;
  if (mixed) {
    // separate instantiations: the mixed path needs far fewer registers
    if (rpw == 1)
      hipLaunchKernelGGL((k_batch_step<1, true, 1>), dim3(g), dim3(kRowThreads), 0, s, probs,
                         row0, nact, step & 1, step % 3);
    else if (rpw == 2)
      hipLaunchKernelGGL((k_batch_step<1, true, 2>), dim3(g), dim3(kRowThreads), 0, s, probs,
                         row0, nact, step & 1, step % 3);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
#define L_(N)                                                                          \
  hipLaunchKernelGGL((k_batch_step<N, false>), dim3(g), dim3(kRowThreads), 0, s, probs, row0, \
                     nact, step & 1, step % 3)
  switch (npl) {
    case 1: L_(1); break;
    case 2: L_(2); break;
    case 4: L_(4); break;
    case 8: L_(8); break;
    case 16: L_(16); break;
    case 32: L_(32); break;
    default: return hipErrorInvalidValue;
  }
#undef L_
  return hipGetLastError();
}

hipError_t launch_rform_step(const ProbDev& P, int npl, int step, hipStream_t s) {
  (void)npl;
  hipLaunchKernelGGL(k_rform_step, dim3((P.nd + kRRows - 1) / kRRows), dim3(256), 0, s, P,
                     step & 1, step % 3);
  return hipGetLastError();
}

hipError_t launch_rform_score(const ProbDev& P, hipStream_t s) {
  hipLaunchKernelGGL(k_rform_score, dim3((P.nd + 255) / 256), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_rform_ut(const ProbDev& P, int f, int kp, z64* Ut, hipStream_t s) {
  if (kp <= 0) return hipSuccess;
  const size_t n = size_t(P.nd) * kp;
  hipLaunchKernelGGL(k_rform_ut, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, P, f, kp, Ut);
  return hipGetLastError();
}

hipError_t launch_rform_t0_init(const ProbDev& P, int f, hipStream_t s) {
  hipLaunchKernelGGL(k_rform_t0_init, dim3((P.nd + 255) / 256, P.nd), dim3(256), 0, s, P, f);
  return hipGetLastError();
}

hipError_t launch_fold_q(const ProbDev& P, int f, int kp, hipStream_t s) {
  if (kp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_q, dim3((P.nd + 255) / 256), dim3(256), 0, s, P, f, kp);
  return hipGetLastError();
}

}  // namespace pngf
