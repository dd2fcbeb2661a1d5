// Device-visible state and argument blocks of the libpngf hot path.
#pragma once

#include "dev_common.h"

namespace pngf {

// DBS bookkeeping kept in device memory so that a whole search runs without
// host round trips (written by the select/prep kernel, read by the others).
struct DbsState {
  int32_t m;           // pixel being accepted by the pending update, -1 none
  int32_t done;        // search finished
  int32_t cursor_s;    // current sweep
  int32_t cursor_pos;  // next position to visit in the current sweep
  int32_t n_acc;       // accepted flips so far
  int32_t sweeps;      // sweeps started
  int32_t converged;   // a whole sweep kept nothing
  int32_t n_sweeps;    // sweep cap of this run
  int64_t attempts;    // visited positions
  uint32_t key;        // min over improving candidates (atomicMin target)
  int32_t pad0;
  double f;            // current objective
  double eta;          // acceptance threshold
  z64 x[kMaxFreq];     // current outputs per frequency
  z64 alpha[kMaxFreq]; // k0^2 delta / den of the pending update
  z64 Em[kMaxFreq];    // E[m] before the pending update
  z64 Rpm[kMaxFreq];   // R'[m] before the pending update
  // mixed precision
  uint32_t key_maybe;  // min key over candidates inside the FP32 error band
  int32_t need_refresh;  // 1: stop and re-form C^-1 in FP64 (2: band hit)
  int32_t n_since;     // accepts since the last FP64 re-inversion
  int32_t kpanel;      // deferred Sherman-Morrison terms held in the panel
  int32_t kslot;       // panel slot of the pending update
  int32_t exact;       // current scores come from the FP64 state
  int64_t n_band;      // decisions that needed the FP64 state
  int32_t flips;       // updates since the buffers were last normalized
                       // (odd: the current vectors/matrix live in the B set)
  int32_t pad1;
  double f_start;      // objective when the current search started
};

// Optional index maps of a complex GEMM (nullptr = identity):
//   A[i][k] = A'[ra[i]][ca[k]],  B[k][n] = B'[rb[k]][cb[n]] (transposed form:
//   B[k][n] = R[rb[n]][cb[k]]),  C'[rc[i]][cc[n]] receives C[i][n].
struct GemmIdx {
  const int32_t *ra = nullptr, *ca = nullptr, *rb = nullptr, *cb = nullptr;
  const int32_t *rc = nullptr, *cc = nullptr;
};

// Partitions of the unpivoted inversion's residual-check maxima (four words
// each: the rows' workgroups spread their atomics over them).
constexpr int kResidParts = 16;

// Workspace of the unpivoted blocked inversion (one per frequency): the
// reduced panels of two consecutive panels (n_S x kNpNb each, row stride
// kNpNb), the pivot rows of the current panel (kNpNb x ld), the inverse of
// its diagonal block (kNpNb x kNpNb), the probe product y (n_S) and three
// maxima of the residual check.
constexpr int kNpNb = 64;
struct NpWork {
  z64* Pt[2];
  z64* X;
  z64* Bi;
  z64* y;
  unsigned long long* mx;
  double tol;   // relative probe residual above which the result is rejected
  const int32_t* rowmap;   // row of the working matrix for each pixel (S rows, then Z rows)
};

// The diagonal tile that a GEMM of the unpivoted inversion inverts once its
// 64 x 64 output tile (tile, tile) is done: block rows and columns
// [k0, k0 + nb) into Bi, a zero pivot flagged in *status (tile < 0: none).
struct NpDiag {
  int tile = -1, k0 = 0, nb = 0;
  z64* Bi = nullptr;
  int32_t* status = nullptr;
};

// One output of a two-product GEMV pass:
//   y[i] = beta w[i] + gamma w2[i] + alpha sum_j A[i,j] d_j v[j].
struct GemvOut {
  const z64* v;
  z64 alpha, beta;
  const z64* w;
  double gamma;
  const z64* w2;
  z64* y;
};

// Everything a hot-path kernel needs, passed by value (kernel arguments).
struct ProbDev {
  int32_t nd, ld, nfreq, max_acc;
  double deps;                 // eps_hi - eps_lo
  double k0sq[kMaxFreq];       // k0^2 per frequency
  double coef[kMaxFreq];       // 1 / (nfreq * norm_f)
  z64* G[kMaxFreq];            // nd x ld, symmetric
  z64* Cinv[kMaxFreq];         // nd x ld, current inverse
  z64* E[kMaxFreq];            // design field
  z64* Rp[kMaxFreq];           // output row R'
  z64* tau[kMaxFreq];          // (C^-1 G)[i,i] at the current state
  z64* q[kMaxFreq];            // copy of C^-1[m,:] for the pending update
  uint8_t* bits;               // design
  const int32_t* perm;         // [n_sweeps][nd] visiting orders
  const int32_t* rank;         // [n_sweeps][nd] position of pixel in order
  int32_t* log_pix;            // [max_acc]
  double* log_f;               // [max_acc]
  double* df;                  // per-candidate objective change (scoring)
  DbsState* st;
  // mixed precision (complex FP32 matrices and the deferred panel)
  z32* C0[kMaxFreq];           // C0^-1 (complex FP32), nd x ld
  z32* G32[kMaxFreq];          // G (complex FP32), nd x ld
  z32* Pp[kMaxFreq];           // panel p vectors, slot k at Pp + k*ld
  z32* Qp[kMaxFreq];           // panel q vectors, slot k at Qp + k*ld
  z64* alph[kMaxFreq];         // alpha of each panel slot
  z64* pcoef[kMaxFreq];        // alpha_k p_k[m] for the pending update
  double* df32;                // FP32-path score of each candidate
  double* dfb;                 // its error bound (before the band factor)
  int32_t kcap;                // panel capacity
  int32_t k_refresh;           // periodic FP64 re-inversion (0: drift-driven)
  double band;                 // relative FP32 error band of a score
  // second buffer set for the one-kernel-per-step search: a step reads one
  // set and writes the other, so no workgroup reads what another writes
  z64* CinvB[kMaxFreq];
  z64* EB[kMaxFreq];
  z64* RpB[kMaxFreq];
  z64* tauB[kMaxFreq];
  uint8_t* bitsB;
  DbsState* stB;               // state of odd steps
  uint32_t* keys;              // [6]: sure keys in slots 0-2, band keys in 3-5
  int32_t* pm;                 // pixel of each panel slot (mixed, R-form)
  // R-form: T0 = C^-1 G at the run start (nd x ld, symmetric) and the FP64
  // panel of columns p_k = T[:, m_k], slot k at Up + k*ld
  z64* T0[kMaxFreq];
  z64* Up[kMaxFreq];
};

}  // namespace pngf
