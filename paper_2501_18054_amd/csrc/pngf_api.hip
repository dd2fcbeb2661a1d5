// C ABI of libpngf: handles, workspace binding and the device-side DBS driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dev_state.h"
#include "pngf_internal.h"

struct pngf_model;

constexpr int kFeatChannels = 7;

namespace pngf {
hipError_t launch_score_rows(const ProbDev& P, int npl, const int32_t* cand, int ncand,
                             uint32_t* keyp, hipStream_t s);
hipError_t launch_plain_step(const ProbDev& P, int npl, int step, hipStream_t s);
hipError_t launch_mixed_step(const ProbDev& P, int npl, int step, hipStream_t s);
hipError_t launch_mixed_persist(const ProbDev& P, int t0, int nsteps, uint64_t* bar,
                                int32_t* flag, int spin_limit, const double* bandp,
                                const int32_t* wstat, hipStream_t s);
hipError_t launch_fold_q(const ProbDev& P, int f, int kp, hipStream_t s);
hipError_t launch_batch_step(const ProbDev* probs, const int32_t* row0, const int32_t* nact,
                             int total, int grid, int npl, int mixed, int rpw, int step,
                             hipStream_t s);
hipError_t launch_accept_only(const ProbDev& P, int npl, hipStream_t s);
hipError_t launch_gemv2(const z64* A, int ld, int n, const uint8_t* bits, double ds,
                        const GemvOut& o1, const GemvOut& o2, hipStream_t s);
hipError_t launch_gemv2_tau(const z64* A, const z64* G, int ld, int n, const GemvOut& o1,
                            const GemvOut& o2, z64* tau, hipStream_t s);
hipError_t launch_score_tail(const ProbDev& P, uint32_t* keyp, hipStream_t s);
hipError_t launch_refresh_tail(const ProbDev& P, const z64* god, z64 xb, uint32_t* keyp,
                               const double* df32, const double* dfb, double* out, double* bandp,
                               const int32_t* gate, hipStream_t s);
hipError_t launch_zgemm(int M, int N, int K, const z64* A, int lda, const int32_t* ca,
                        const z64* B, int ldb, bool transb, const int32_t* rb, z64* C, int ldc,
                        z64 alpha, z64 beta, int splits, z64* work, hipStream_t s,
                        int* nz_out = nullptr);
hipError_t launch_rform_step(const ProbDev& P, int npl, int step, hipStream_t s);
hipError_t launch_rform_score(const ProbDev& P, hipStream_t s);
hipError_t launch_rform_ut(const ProbDev& P, int f, int kp, z64* Ut, hipStream_t s);
hipError_t launch_rform_t0_init(const ProbDev& P, int f, hipStream_t s);
hipError_t launch_wood_cap(z64* P, int ldp, int nd, const int32_t* F, int k, const double* sc,
                           z64* Cap, int32_t* status, hipStream_t s,
                           const int32_t* kdev = nullptr);
hipError_t launch_small_inverse(z64* A, int k, int32_t* status, hipStream_t s);
hipError_t launch_wood_panel(const z64* work, int nz, int nd, int k, const double* sc, z64* P,
                             int ldp, const int32_t* F, z64* Cap, int32_t* status, hipStream_t s,
                             const int32_t* kdev = nullptr);
hipError_t launch_wood_prep(const ProbDev& P, uint8_t* bref, int kpad, int32_t* dF,
                            double* dS, int32_t* wk, hipStream_t s);
hipError_t launch_gradient(const ProbDev& P, double* out, hipStream_t s);
hipError_t launch_tile_score(const ProbDev& P, const int32_t* tiles, int ntiles, int m, int ks,
                             z64* part, double* out, hipStream_t s);
int tile_rows(int m);
hipError_t launch_pick_best(const double* df, const int32_t* cand, int n, const DbsState* st,
                            int32_t* out, hipStream_t s);
hipError_t model_score_state(pngf_model* m, const ProbDev& P, float** scores);
hipError_t launch_rank(const float* s, int n, int32_t* out, hipStream_t st);
hipError_t launch_features(const ProbDev& P, int H, int W, float* X, hipStream_t s);
hipError_t launch_ranked_keys(const ProbDev& P, const float* score, DbsState* st, int src,
                              uint32_t* key_sure, uint32_t* key_band, hipStream_t s);
int model_hw(pngf_model* m, int* H, int* W);
hipStream_t model_stream(pngf_model* m);
hipError_t launch_select_prep(const ProbDev& P, int forced, hipStream_t s);
hipError_t launch_segment_start(const ProbDev& P, int reset_panel, hipStream_t s);
hipError_t launch_state_begin(DbsState* st, int n_sweeps, double eta, hipStream_t s);
hipError_t launch_accept_rescore(const ProbDev& P, int npl, hipStream_t s);
hipError_t launch_inverse(z64* S, z64* Cinv, const z64* G, int nd, int ld, const int32_t* sidx,
                          const int32_t* zidx, const int32_t* pos, int ns, double k2d, z64* B1,
                          z64* Pb, z64* Pn, int32_t* piv, int32_t* inv_p, int32_t* used,
                          int32_t* status, int32_t* tsbuf, z64* B11inv, const NpWork* np,
                          hipStream_t s);
hipError_t launch_gemv(const z64* A, int ld, int n, const z64* v, const uint8_t* bits, double ds,
                       z64 alpha, z64 beta, const z64* w, double gamma, const z64* w2, z64* y,
                       hipStream_t s, z32* A32 = nullptr);
hipError_t launch_output(const ProbDev& P, int f, const z64* god, z64 xb, int last,
                         hipStream_t s);
hipError_t launch_to_c64(const z64* src, z32* dst, int nd, int ld, hipStream_t s);
hipError_t launch_fold(const ProbDev& P, int f, int kp, hipStream_t s);
hipError_t launch_band_measure(const double* df32, const double* bnd32, const double* df64,
                               int nd, double* out, const int32_t* status, hipStream_t s,
                               double* bandp = nullptr, const int32_t* gate = nullptr);
constexpr int kGjNbHost = 16;
constexpr int kPanelCap = 64;      // deferred Sherman-Morrison terms (mixed)
constexpr int kMixedBatch = 16;    // device steps between host checks (mixed)
constexpr int kPersistBatch = 32;  // steps of one persistent launch (periodic refresh)
constexpr int kPersistSpin = 1 << 20;   // polls of a persistent-search grid barrier
constexpr int kPersistSlotsHost = 64;   // panel slots the persistent search holds in LDS
constexpr int kPersistBarWords = 2 * 16 * 18;   // grid-barrier words (as int32) of the persistent search
constexpr size_t kPersistBarBytes = (kPersistBarWords + 32) * sizeof(int32_t);
constexpr size_t kPinBytes = 16384;          // pinned scratch of small transfers
constexpr size_t kPinUpload = 256;           // offset of the Woodbury upload in it
constexpr size_t kPinState = 8192;           // offset of a search's state read
constexpr size_t kStageOrders = 1024;        // visiting orders in the staging area, after the state
static_assert(kPinUpload + 256 + kMaxFreq * 64 * sizeof(double) <= kPinState &&
                  kPinState + sizeof(DbsState) <= kPinBytes,
              "pinned scratch regions overlap");
constexpr size_t kPinBand = 32;             // the error band a search starts from
constexpr size_t kPinInvStatus = 64;        // status of an initial inverse checked later
// the small slots: band measurement {max, status} at 8, a Woodbury status at
// 24, then the band and the inverse status, all below the Woodbury upload
static_assert(kPinBand >= 28 && kPinBand + sizeof(double) <= kPinInvStatus &&
                  kPinInvStatus + sizeof(int32_t) <= kPinUpload,
              "pinned scratch slots overlap");
constexpr size_t kPinStage = kPinBytes;      // then the batch-end read (state .. bits), then
                                             // the index lists of an initial inverse
constexpr double kDriftTol = 1e-5; // relative FP64 residual of E that forces a re-inversion
constexpr int kWoodMax = 64;       // flips folded by one FP64 block-Woodbury refresh
constexpr int kBatchRefreshStreams = 4;   // streams a batch spreads one round's refreshes over
constexpr int kAheadMaxK = 32;   // largest k_refresh whose refreshes are queued ahead of the host
constexpr int kTilePartPerPixel = 512;   // tile-score partial blocks (complex) per pixel
constexpr int kTileSlicesMax = 32;       // K slices of one tile's block
constexpr int kWoodSplits = 8;     // split-K factor of its skinny GEMM
constexpr int kRPanel = 512;       // R-form panel capacity before a fold into T0
constexpr int kDriftEvery = 32;    // accepts between drift checks
}  // namespace pngf

using pngf::cd;
using pngf::z32;
using pngf::z64;

namespace {

thread_local std::string g_create_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

enum KernelId { KID_SCORE = 0, KID_SELECT = 1, KID_ACCEPT = 2, KID_LU = 3, KID_OTHER = 4,
                KID_FOLD = 5, KID_MIXQ = 6, KID_WOOD = 7, KID_TILE = 8, KID_N = 9 };

struct Layout {
  size_t off_G[pngf::kMaxFreq], off_C[pngf::kMaxFreq], off_E[pngf::kMaxFreq],
      off_Rp[pngf::kMaxFreq], off_tau[pngf::kMaxFreq], off_q[pngf::kMaxFreq];
  size_t off_b[pngf::kMaxFreq], off_god[pngf::kMaxFreq];
  size_t off_bits, off_perm, off_rank, off_cand, off_df, off_logp, off_logf, off_state;
  size_t off_C0[pngf::kMaxFreq], off_G32[pngf::kMaxFreq], off_Pp[pngf::kMaxFreq],
      off_Qp[pngf::kMaxFreq], off_alph[pngf::kMaxFreq], off_pcoef[pngf::kMaxFreq];
  size_t off_df32, off_dfb, off_bandout, off_bref, off_wk;
  size_t off_sidx, off_zidx, off_pos, off_rowmap;
  size_t off_CB[pngf::kMaxFreq], off_EB[pngf::kMaxFreq], off_RpB[pngf::kMaxFreq],
      off_tauB[pngf::kMaxFreq];
  size_t off_bitsB, off_stateB, off_keys, off_pm, off_best, off_feat;
  // inversion and block-Woodbury workspaces, one set per frequency (the
  // frequencies' systems are independent and run on their own streams)
  size_t off_S[pngf::kMaxFreq], off_B1[pngf::kMaxFreq], off_Pb[pngf::kMaxFreq],
      off_Pn[pngf::kMaxFreq], off_ts[pngf::kMaxFreq], off_B11[pngf::kMaxFreq],
      off_piv[pngf::kMaxFreq], off_invp[pngf::kMaxFreq], off_used[pngf::kMaxFreq],
      off_np[pngf::kMaxFreq];
  size_t off_status, off_pbar, off_flag, off_band, off_u[pngf::kMaxFreq], off_r[pngf::kMaxFreq];
  size_t off_wP[pngf::kMaxFreq], off_wW[pngf::kMaxFreq],
      off_wCap[pngf::kMaxFreq], off_wWork[pngf::kMaxFreq];
  size_t off_wF, off_wS, off_tiles, off_tpart;
  size_t off_T[pngf::kMaxFreq], off_Up[pngf::kMaxFreq], off_ralph[pngf::kMaxFreq], off_rpm, off_Ut;
  size_t total;
};

}  // namespace

struct pngf_handle {
  pngf::Precomputed pc;
  std::string err;
  pngf_options opt{};
  bool bound = false;
  bool have_design = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int ld = 0, npl = 1;
  bool persist_off = false;   // a launch of the persistent search was refused
  // ranked search: the visiting order of every state is a fresh ranking of
  // the pixels (by rank_model, or by the first-order change if it is null)
  bool ranked = false;
  pngf_model* rank_model = nullptr;
  int rank_h = 0, rank_w = 0;
  int persist_spin = pngf::kPersistSpin;   // polls of one grid-barrier wait
  double np_tol = 1e-12;           // probe-residual bound of the unpivoted inversion
  int64_t n_inv_np = 0, n_inv_piv = 0;   // inversions by each path
  bool reform_c64 = false;   // reform_fields also writes C0^-1 (mixed refresh)
  bool persist_ok = false;   // a persistent launch of this search has run
  bool persist_aborted = false;   // the last one found a pending refresh singular
  int force_singular = 0;   // block-Woodbury refreshes still to report singular (test hook)
  Layout lay{};
  pngf::ProbDev P{};
  std::vector<uint8_t> bits;
  std::vector<uint8_t> bits_ref;   // design whose FP64 inverse C^-1 holds (mixed runs)
  bool cinv_stale = false;         // an R-form search moved the design past C^-1
  // host copy of the design read with the last batch of steps (saves a
  // round trip before the next FP64 refresh), and the host arrays a deferred
  // block-Woodbury update copies from (kept until its wait)
  bool bits_fresh = false;
  char* pin = nullptr;             // pinned scratch of small transfers, then a staging area
  size_t pin_bytes = 0;
  hipEvent_t ev_pin = nullptr;     // recorded after the last upload from `pin`
  hipEvent_t ev_ahead = nullptr;   // after a batch's state read, ahead of its refresh
  // an initial inverse queued by set_design and not yet checked: its status
  // lands at pin + kPinInvStatus, ev_inv is recorded after that read, and its
  // index lists go up from pin + pin_idx (a region nothing else writes)
  bool inv_pending = false;
  hipEvent_t ev_inv = nullptr;
  size_t pin_idx = 0;
  std::vector<int32_t> w_fl;
  std::vector<double> w_sc;
  bool wood_pending = false;       // a Woodbury status not yet read
  bool rescore_pending = false;    // refresh_rescore queued a read of that status
  bool tau_fresh = false;          // the last fp64_refresh formed every candidate's tau
  double f_host = 0.0;
  // event timing
  double ktime_ms[KID_N] = {0};
  int64_t klaunch[KID_N] = {0};
  std::vector<hipEvent_t> ev_pool;   // recorded (start, end, kernel id) triples
  std::vector<hipEvent_t> ev_free;   // created events ready for reuse
  int32_t nacc_seen = 0;             // accepts counted by the step timing so far
  // streams of frequencies 1..F-1 for per-frequency work (default priority),
  // with the events that fork them from and join them to the bound stream
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
};

namespace {

int fail(pngf_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

#define HIPCHK(h, call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return fail(h, PNGF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int npl_for(int nd) {
  int need = (nd + pngf::kRowThreads - 1) / pngf::kRowThreads;
  int n = 1;
  while (n < need) n *= 2;
  return n;
}

Layout make_layout(const pngf_handle* h, const pngf_options* o) {
  Layout L{};
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t r = off; off = align256(off + bytes); return r; };
  const size_t mat = size_t(nd) * ld * sizeof(z64), vec = size_t(ld) * sizeof(z64);
  for (int f = 0; f < F; ++f) {
    L.off_G[f] = take(mat);
    L.off_C[f] = take(mat);
    L.off_E[f] = take(vec);
    L.off_Rp[f] = take(vec);
    L.off_tau[f] = take(vec);
    L.off_q[f] = take(vec);
    L.off_b[f] = take(vec);
    L.off_god[f] = take(vec);
    if (o->precision == PNGF_FP64_PLAIN) L.off_CB[f] = take(mat);
    L.off_EB[f] = take(vec);
    L.off_RpB[f] = take(vec);
    L.off_tauB[f] = take(vec);
  }
  L.off_stateB = take(sizeof(pngf::DbsState));
  L.off_keys = take(6 * sizeof(uint32_t));
  L.off_pm = take(size_t(pngf::kPanelCap) * sizeof(int32_t));
  L.off_best = take(4 * sizeof(int32_t));
  L.off_feat = take(size_t(kFeatChannels) * nd * sizeof(float));
  if (o->precision == PNGF_MIXED) {
    const size_t mat32 = size_t(nd) * ld * sizeof(z32);
    for (int f = 0; f < F; ++f) {
      L.off_C0[f] = take(mat32);
      L.off_G32[f] = take(mat32);
      L.off_Pp[f] = take(size_t(pngf::kPanelCap) * ld * sizeof(z32));
      L.off_Qp[f] = take(size_t(pngf::kPanelCap) * ld * sizeof(z32));
      L.off_alph[f] = take(size_t(pngf::kPanelCap) * sizeof(z64));
      L.off_pcoef[f] = take(size_t(pngf::kPanelCap) * sizeof(z64));
    }
    L.off_df32 = take(size_t(nd) * sizeof(double));
    L.off_dfb = take(size_t(nd) * sizeof(double));
    L.off_bandout = take(2 * sizeof(double));
    // a refresh queued ahead of the host: the design of C^-1 on the device,
    // the flip count and the measurement gate
    L.off_bref = take(size_t(nd));
    L.off_wk = take(4 * sizeof(int32_t));
  }
  if (o->precision == PNGF_RFORM) {
    const size_t kr = size_t(pngf::kRPanel);
    for (int f = 0; f < F; ++f) {
      L.off_T[f] = take(mat);
      L.off_Up[f] = take(kr * ld * sizeof(z64));
      L.off_ralph[f] = take(kr * sizeof(z64));
    }
    L.off_rpm = take(kr * sizeof(int32_t));
    L.off_Ut = take(size_t(nd) * kr * sizeof(z64));
  }
  if (o->precision == PNGF_FP64_PLAIN && o->max_tile > 0) {
    L.off_tiles = take(size_t(nd) * o->max_tile * sizeof(int32_t));
    L.off_tpart = take(size_t(nd) * pngf::kTilePartPerPixel * sizeof(z64));
  }
  {
    // FP64 block-Woodbury update (mixed refresh, tile accept, pixel sets):
    // panel, rows, capacitance, split-K partials
    const size_t kw = size_t(pngf::kWoodMax);
    for (int f = 0; f < F; ++f) {
      L.off_wP[f] = take(size_t(nd) * kw * sizeof(z64));
      L.off_wW[f] = take(kw * nd * sizeof(z64));
      L.off_wCap[f] = take(kw * kw * sizeof(z64));
      L.off_wWork[f] = take(size_t(pngf::kWoodSplits) * nd * kw * sizeof(z64));
    }
    L.off_wF = take(kw * sizeof(int32_t));
    L.off_wS = take(size_t(F) * kw * sizeof(double));
  }
  for (int f = 0; f < F; ++f) {
    L.off_S[f] = take(mat);
    L.off_B1[f] = take(2 * size_t(pngf::kGjNbHost) * ld * sizeof(z64));
    L.off_Pb[f] = take(size_t(pngf::kGjNbHost) * ld * sizeof(z64));
    L.off_Pn[f] = take(size_t(pngf::kGjNbHost) * ld * sizeof(z64));
    // tournament: an arrival count, then two proposal lists of (kGjNb + 1)
    // ints per 64-row group
    L.off_ts[f] = take(256 + size_t(2) * (pngf::kGjNbHost + 1) * ((nd + 63) / 64) * sizeof(int32_t));
    L.off_B11[f] = take(size_t(pngf::kGjNbHost) * pngf::kGjNbHost * sizeof(z64));
    L.off_piv[f] = take(size_t(nd) * sizeof(int32_t));
    L.off_invp[f] = take(size_t(nd) * sizeof(int32_t));
    L.off_used[f] = take(size_t(nd) * sizeof(int32_t));
    // unpivoted inversion: two reduced panels, the pivot rows, the block
    // inverse, the probe product and the check's maxima
    L.off_np[f] = take((3 * size_t(pngf::kNpNb) * ld + size_t(pngf::kNpNb) * pngf::kNpNb + nd) *
                           sizeof(z64) + 4 * pngf::kResidParts * sizeof(unsigned long long));
  }
  L.off_sidx = take(size_t(nd) * sizeof(int32_t));
  L.off_zidx = take(size_t(nd) * sizeof(int32_t));
  L.off_pos = take(size_t(nd) * sizeof(int32_t));
  L.off_rowmap = take(size_t(nd) * sizeof(int32_t));
  L.off_status = take(sizeof(int32_t));
  L.off_band = take(sizeof(double));   // the error band as the device holds it
  L.off_pbar = take(pngf::kPersistBarBytes);   // grid-barrier words, then the time-out flag
  for (int f = 0; f < F; ++f) {
    L.off_u[f] = take(vec);
    L.off_r[f] = take(vec);
  }
  const int ms = std::max(1, o->max_sweeps), ma = std::max(1, o->max_accepts);
  L.off_perm = take(size_t(ms) * nd * sizeof(int32_t));
  L.off_rank = take(size_t(ms) * nd * sizeof(int32_t));
  L.off_cand = take(size_t(nd) * sizeof(int32_t));
  L.off_df = take(size_t(nd) * sizeof(double));
  L.off_logp = take(size_t(ma) * sizeof(int32_t));
  L.off_logf = take(size_t(ma) * sizeof(double));
  // adjacent, so that one copy brings them to the host after a batch of steps
  L.off_state = take(sizeof(pngf::DbsState));
  L.off_flag = take(sizeof(int32_t));
  L.off_bits = take(size_t(nd));
  L.off_bitsB = take(size_t(nd));
  L.total = off;
  return L;
}

template <class T>
T* at(pngf_handle* h, size_t off) { return reinterpret_cast<T*>(h->ws + off); }

int settle_inverse(pngf_handle* h, bool* redone = nullptr);

// A bound handle (with a design if need_design; its initial inverse then
// checked, unless settle is false and the caller checks it later).
int check_ready(pngf_handle* h, bool need_design, bool settle = true) {
  if (!h) return PNGF_EINVAL;
  if (!h->bound) return fail(h, PNGF_ESTATE, "handle is not bound to a workspace");
  if (need_design && !h->have_design) return fail(h, PNGF_ESTATE, "no design set");
  if (need_design && settle) return settle_inverse(h);
  return PNGF_OK;
}

hipStream_t fstream(pngf_handle* h, int f) { return f == 0 ? h->stream : h->aux[f - 1]; }

// Make the frequency streams wait for the work queued so far on the bound
// stream, and the bound stream for everything the frequency streams queue.
int fork_streams(pngf_handle* h) {
  if (h->aux.empty()) return PNGF_OK;
  HIPCHK(h, hipEventRecord(h->ev_fork, h->stream));
  for (hipStream_t a : h->aux) HIPCHK(h, hipStreamWaitEvent(a, h->ev_fork, 0));
  return PNGF_OK;
}

int join_streams(pngf_handle* h) {
  for (size_t k = 0; k < h->aux.size(); ++k) {
    HIPCHK(h, hipEventRecord(h->ev_join[k], h->aux[k]));
    HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_join[k], 0));
  }
  return PNGF_OK;
}

void release_streams(pngf_handle* h) {
  for (hipStream_t a : h->aux) (void)hipStreamDestroy(a);
  for (hipEvent_t e : h->ev_join) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  h->aux.clear();
  h->ev_join.clear();
  h->ev_fork = nullptr;
}

// Timed launch helper: records events around the launch when timing is on.
struct Timer {
  pngf_handle* h;
  int kid;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t take(pngf_handle* h) {
    hipEvent_t e = nullptr;
    if (!h->ev_free.empty()) {
      e = h->ev_free.back();
      h->ev_free.pop_back();
    } else {
      hipEventCreate(&e);
    }
    return e;
  }
  Timer(pngf_handle* hh, int k) : h(hh), kid(k) {
    if ((h->opt.flags & PNGF_FLAG_TIMING) ||
        ((h->opt.flags & PNGF_FLAG_TIMING_STEPS) && kid == KID_ACCEPT)) {
      a = take(h);
      b = take(h);
      hipEventRecord(a, h->stream);
    }
  }
  // count: launches of the kernel class between the two events
  void end(int count = 1) {
    if (a) {
      hipEventRecord(b, h->stream);
      h->ev_pool.push_back(a);
      h->ev_pool.push_back(b);
      h->ev_pool.push_back(reinterpret_cast<hipEvent_t>(intptr_t(kid) | (intptr_t(count) << 8)));
    }
  }
};
void collect_times(pngf_handle* h) {
  for (size_t k = 0; k + 2 < h->ev_pool.size() + 0; k += 3) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, h->ev_pool[k], h->ev_pool[k + 1]);
    const intptr_t tag = reinterpret_cast<intptr_t>(h->ev_pool[k + 2]);
    const int kid = int(tag & 0xFF);
    h->ktime_ms[kid] += ms;
    h->klaunch[kid] += int64_t(tag >> 8);
    h->ev_free.push_back(h->ev_pool[k]);
    h->ev_free.push_back(h->ev_pool[k + 1]);
  }
  h->ev_pool.clear();
}

// E = C^-1 b with one step of FP64 iterative refinement against C, then
// R' = G_OD (I + k0^2 D C^-1 G) = G_OD + k0^2 C^-1 (G D G_OD) (reciprocity)
// and the outputs, for the design in P.bits and the C^-1 in P.Cinv.  With
// tau, the second pass over C^-1 also forms every candidate's tau (reading
// the rows of G beside those of C^-1), for k_score_tail.  Without output the
// outputs x and f are left to the caller (k_refresh_tail).
int reform_fields(pngf_handle* h, bool tau = false, bool output = true) {
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  const Layout& L = h->lay;
  pngf::ProbDev& P = h->P;
  const z64 one{1.0, 0.0}, zero{0.0, 0.0};
  // sequential on the bound stream: each GEMV pass already spans the chip
  // (frequency streams measured slower here than in order)
  for (int f = 0; f < F; ++f) {
    const double k2 = P.k0sq[f];
    const z64* b = at<z64>(h, L.off_b[f]);
    const z64* god = at<z64>(h, L.off_god[f]);
    z64* u = at<z64>(h, L.off_u[f]);
    z64* r = at<z64>(h, L.off_r[f]);
    Timer t(h, KID_OTHER);
    // E = C^-1 b (and, for a mixed refresh, C0^-1 = complex-FP32 C^-1 from
    // the same pass)
    HIPCHK(h, pngf::launch_gemv(P.Cinv[f], ld, nd, b, nullptr, 0.0, one, zero, nullptr, 0.0,
                                nullptr, P.E[f], h->stream, h->reform_c64 ? P.C0[f] : nullptr));
    // one pass over G:  r = b - E + k0^2 G diag(deps) E,  u = G diag(deps) G_OD
    const pngf::GemvOut o_r{P.E[f], z64{k2, 0.0}, one, b, -1.0, P.E[f], r};
    const pngf::GemvOut o_u{god, one, zero, nullptr, 0.0, nullptr, u};
    HIPCHK(h, pngf::launch_gemv2(P.G[f], ld, nd, P.bits, P.deps, o_r, o_u, h->stream));
    // one pass over C^-1:  E += C^-1 r,  R' = G_OD + k0^2 C^-1 u
    const pngf::GemvOut o_e{r, one, one, P.E[f], 0.0, nullptr, P.E[f]};
    const pngf::GemvOut o_p{u, z64{k2, 0.0}, one, god, 0.0, nullptr, P.Rp[f]};
    if (tau)
      HIPCHK(h, pngf::launch_gemv2_tau(P.Cinv[f], P.G[f], ld, nd, o_e, o_p, P.tau[f], h->stream));
    else
      HIPCHK(h, pngf::launch_gemv2(P.Cinv[f], ld, nd, nullptr, 0.0, o_e, o_p, h->stream));
    const cd xb = h->pc.freq[f].xb;
    if (output)
      HIPCHK(h, pngf::launch_output(P, f, god, z64{xb.real(), xb.imag()}, f == F - 1, h->stream));
    t.end();
  }
  return PNGF_OK;
}

// The unpivoted inversion's workspace of frequency f.
pngf::NpWork np_work(pngf_handle* h, int f) {
  const size_t ld = size_t(h->ld), nb = size_t(pngf::kNpNb);
  z64* base = at<z64>(h, h->lay.off_np[f]);
  pngf::NpWork w;
  w.Pt[0] = base;
  w.Pt[1] = base + nb * ld;
  w.X = base + 2 * nb * ld;
  w.Bi = base + 3 * nb * ld;
  w.y = w.Bi + nb * nb;
  w.mx = reinterpret_cast<unsigned long long*>(w.y + h->pc.n_d);
  w.tol = h->np_tol;
  w.rowmap = at<int32_t>(h, h->lay.off_rowmap);
  return w;
}

// Re-form C^-1 (FP64, on the device) from G and the device design bits for
// every frequency, then E, R', x and f (reform_fields).
// host_bits: h->bits already holds the device design (no read back).  The
// fields are re-formed before the inversion's status is read (one wait for
// both; the rare rejected result is re-formed again after the pivot search).
// With defer (no kernel timing), the unpivoted result is not waited for: its
// status goes to pinned memory behind an event, and settle_inverse checks it
// when the handle is next used.  pivot_only skips the unpivoted attempt.
int device_reinvert(pngf_handle* h, bool host_bits = false, bool defer = false,
                    bool pivot_only = false) {
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  const Layout& L = h->lay;
  pngf::ProbDev& P = h->P;
  if (h->inv_pending) {
    // a queued initial inverse this one replaces: its index-list copies must
    // have run before the region is written again (it counts as an
    // unpivoted inversion if it passed its check)
    HIPCHK(h, hipEventSynchronize(h->ev_inv));
    h->inv_pending = false;
    if (*reinterpret_cast<const int32_t*>(h->pin + pngf::kPinInvStatus) == 0) ++h->n_inv_np;
  }
  int32_t* status = at<int32_t>(h, L.off_status);
  HIPCHK(h, hipMemsetAsync(status, 0, sizeof(int32_t), h->stream));
  // S (pixels at eps_hi) and Z from the device design bits
  if (!host_bits) {
    HIPCHK(h, hipMemcpyAsync(h->bits.data(), P.bits, nd, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  std::vector<int32_t> sidx, zidx, pos(nd, -1), rowmap(nd);
  for (int i = 0; i < nd; ++i) {
    if (h->bits[i]) { pos[i] = int32_t(sidx.size()); sidx.push_back(i); }
    else zidx.push_back(i);
  }
  const int ns = int(sidx.size());
  // the unpivoted inversion's working matrix: S rows, then Z rows
  for (int i = 0, z = 0; i < nd; ++i) rowmap[i] = pos[i] >= 0 ? pos[i] : ns + z++;
  int32_t* d_sidx = at<int32_t>(h, L.off_sidx);
  int32_t* d_zidx = at<int32_t>(h, L.off_zidx);
  int32_t* d_pos = at<int32_t>(h, L.off_pos);
  // the index lists go up from their own pinned region (written again only
  // after this inversion's event, see above)
  auto* stg = reinterpret_cast<int32_t*>(h->pin + h->pin_idx);
  std::copy(sidx.begin(), sidx.end(), stg);
  std::copy(zidx.begin(), zidx.end(), stg + ns);
  std::copy(pos.begin(), pos.end(), stg + nd);
  std::copy(rowmap.begin(), rowmap.end(), stg + 2 * nd);
  const int32_t* src_s = stg;
  const int32_t* src_z = stg + ns;
  const int32_t* src_p = stg + nd;
  const int32_t* src_m = stg + 2 * nd;
  if (ns > 0)
    HIPCHK(h, hipMemcpyAsync(d_sidx, src_s, ns * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  if (nd - ns > 0)
    HIPCHK(h, hipMemcpyAsync(d_zidx, src_z, (nd - ns) * sizeof(int32_t), hipMemcpyHostToDevice,
                             h->stream));
  HIPCHK(h, hipMemcpyAsync(d_pos, src_p, nd * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(at<int32_t>(h, L.off_rowmap), src_m, nd * sizeof(int32_t),
                           hipMemcpyHostToDevice, h->stream));
  // one inversion per frequency, each on its own stream; first without row
  // exchanges, and with the pivot search where that result fails its check
  // (or always, with PNGF_FLAG_PIVOT_SEARCH)
  const bool force_piv = (h->opt.flags & PNGF_FLAG_PIVOT_SEARCH) != 0;
  for (int pass = (force_piv || pivot_only) ? 1 : 0; pass < 2; ++pass) {
    const bool pivoted = pass == 1;
    if (pivoted && !force_piv && !pivot_only)
      HIPCHK(h, hipMemsetAsync(status, 0, sizeof(int32_t), h->stream));
    {
      Timer t(h, KID_LU);
      int st = fork_streams(h);
      if (st) return st;
      for (int f = 0; f < F; ++f) {
        const pngf::NpWork np = np_work(h, f);
        HIPCHK(h, pngf::launch_inverse(at<z64>(h, L.off_S[f]), P.Cinv[f], P.G[f], nd, ld, d_sidx,
                                       d_zidx, d_pos, ns, P.k0sq[f] * P.deps,
                                       at<z64>(h, L.off_B1[f]), at<z64>(h, L.off_Pb[f]),
                                       at<z64>(h, L.off_Pn[f]), at<int32_t>(h, L.off_piv[f]),
                                       at<int32_t>(h, L.off_invp[f]),
                                       at<int32_t>(h, L.off_used[f]), status,
                                       at<int32_t>(h, L.off_ts[f]), at<z64>(h, L.off_B11[f]),
                                       pivoted ? nullptr : &np, fstream(h, f)));
      }
      st = join_streams(h);
      if (st) return st;
      t.end(F);
    }
    int st = reform_fields(h);
    if (st) return st;
    if (defer && !pivoted && !(h->opt.flags & PNGF_FLAG_TIMING)) {
      auto* sp = reinterpret_cast<int32_t*>(h->pin + pngf::kPinInvStatus);
      HIPCHK(h, hipMemcpyAsync(sp, status, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipEventRecord(h->ev_inv, h->stream));
      h->inv_pending = true;
      h->bits_ref = h->bits;
      h->cinv_stale = false;
      return PNGF_OK;
    }
    int32_t st_host = 0;
    HIPCHK(h, hipMemcpyAsync(&st_host, status, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (!pivoted && (st_host & 2)) continue;
    if (st_host) return fail(h, PNGF_ESINGULAR, "zero pivot while inverting the PNGF system matrix");
    ++(pivoted ? h->n_inv_piv : h->n_inv_np);
    break;
  }
  if (h->opt.flags & (PNGF_FLAG_TIMING | PNGF_FLAG_TIMING_STEPS)) collect_times(h);
  h->bits_ref = h->bits;
  h->cinv_stale = false;
  return PNGF_OK;
}

// The check of an initial inverse that set_design queued without waiting:
// waits for its status, and where the unpivoted result failed its probe
// residual inverts again with the pivot search (*redone then says that the
// fields were formed again, after anything queued since).  A zero pivot
// drops the design.
int settle_inverse(pngf_handle* h, bool* redone) {
  if (redone) *redone = false;
  if (!h->inv_pending) return PNGF_OK;
  h->inv_pending = false;
  HIPCHK(h, hipEventSynchronize(h->ev_inv));
  const int32_t st_host = *reinterpret_cast<const int32_t*>(h->pin + pngf::kPinInvStatus);
  int st = PNGF_OK;
  if (st_host == 0) {
    ++h->n_inv_np;
  } else if (st_host & 2) {
    if (redone) *redone = true;
    st = device_reinvert(h, true, false, true);
  } else {
    st = fail(h, PNGF_ESINGULAR, "zero pivot while inverting the PNGF system matrix");
  }
  if (st) h->have_design = false;
  return st;
}

// Block-Woodbury update of the FP64 inverse in P.Cinv (eq. lru_woodbury,
// M = fl.size() <= kWoodMax) for the pixels fl, whose bits in cur are their
// new values: C^-1 += P W with P = C^-1 G[:,F] diag(k0^2 delta_F) and
// W = Cap^-1 C^-1[F,:], Cap the M x M capacitance matrix, on the matrix
// cores.  *singular reports a singular Cap (C^-1 is then not usable).  Ends
// with a wait.
int woodbury_update(pngf_handle* h, const std::vector<int32_t>& fl, const std::vector<uint8_t>& cur,
                    bool* singular, bool defer = false) {
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  const Layout& L = h->lay;
  pngf::ProbDev& P = h->P;
  const int k = int(fl.size());
  int32_t* dF = at<int32_t>(h, L.off_wF);
  double* dS = at<double>(h, L.off_wS);
  int32_t* status = at<int32_t>(h, L.off_status);
  h->w_fl = fl;
  std::vector<double>& sc = h->w_sc;
  sc.assign(size_t(F) * k, 0.0);
  for (int f = 0; f < F; ++f)
    for (int c = 0; c < k; ++c)
      sc[size_t(f) * k + c] = P.k0sq[f] * (cur[fl[c]] ? P.deps : -P.deps);
  // one frequency: the capacitance kernel clears the status in stream order
  if (F > 1) HIPCHK(h, hipMemsetAsync(status, 0, sizeof(int32_t), h->stream));
  {
    // the flips and scales in one upload through the pinned scratch (laid
    // out like dF .. dS in the workspace), once its previous upload is done
    const size_t gap = L.off_wS - L.off_wF;
    HIPCHK(h, hipEventSynchronize(h->ev_pin));
    int32_t* pf = reinterpret_cast<int32_t*>(h->pin + pngf::kPinUpload);
    double* ps = reinterpret_cast<double*>(h->pin + pngf::kPinUpload + gap);
    std::copy(h->w_fl.begin(), h->w_fl.end(), pf);
    std::copy(sc.begin(), sc.end(), ps);
    HIPCHK(h, hipMemcpyAsync(dF, pf, gap + size_t(F) * k * sizeof(double), hipMemcpyHostToDevice,
                             h->stream));
    HIPCHK(h, hipEventRecord(h->ev_pin, h->stream));
  }
  const z64 one{1.0, 0.0}, zero{0.0, 0.0};
  {
    Timer t(h, KID_WOOD);
    int st = fork_streams(h);
    if (st) return st;
    for (int f = 0; f < F; ++f) {
      const hipStream_t sf = fstream(h, f);
      z64* wP = at<z64>(h, L.off_wP[f]);
      z64* wW = at<z64>(h, L.off_wW[f]);
      z64* cap = at<z64>(h, L.off_wCap[f]);
      // P = C_ref^-1 G[:,F] diag(k0^2 delta_F)   (G[:,F] = G[F,:]^T): split-K
      // partials, then one pass that reduces, scales and forms Cap
      z64* wk = at<z64>(h, L.off_wWork[f]);
      int nzp = 0;
      HIPCHK(h, pngf::launch_zgemm(nd, k, nd, P.Cinv[f], ld, nullptr, P.G[f], ld, true, dF, wP, k,
                                   one, zero, pngf::kWoodSplits, wk, sf, &nzp));
      if (nzp > 0) {
        HIPCHK(h, pngf::launch_wood_panel(wk, nzp, nd, k, dS + size_t(f) * k, wP, k, dF, cap,
                                          F == 1 ? status : nullptr, sf));
      } else {
        HIPCHK(h, pngf::launch_wood_cap(wP, k, nd, dF, k, dS + size_t(f) * k, cap,
                                        F == 1 ? status : nullptr, sf));
      }
      HIPCHK(h, pngf::launch_small_inverse(cap, k, status, sf));
      if (h->force_singular > 0 && f == F - 1) {
        // test hook: this refresh reports a singular capacitance matrix
        HIPCHK(h, hipMemsetAsync(status, 1, sizeof(int32_t), sf));
        --h->force_singular;
      }
      // W = Cap^-1 C_ref^-1[F,:] (the rows F gathered by the GEMM);
      // C^-1 = C_ref^-1 + P W
      HIPCHK(h, pngf::launch_zgemm(k, nd, k, cap, k, nullptr, P.Cinv[f], ld, false, dF, wW, nd,
                                   one, zero, 1, nullptr, sf));
      HIPCHK(h, pngf::launch_zgemm(nd, nd, k, wP, k, nullptr, wW, nd, false, nullptr, P.Cinv[f],
                                   ld, one, one, 1, nullptr, sf));
    }
    st = join_streams(h);
    if (st) return st;
    t.end(F);
  }
  *singular = false;
  if (defer) {
    // the caller reads the status at its next wait (wood_pending)
    h->wood_pending = true;
    return PNGF_OK;
  }
  int32_t st_host = 0;
  HIPCHK(h, hipMemcpyAsync(&st_host, status, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *singular = st_host != 0;
  return PNGF_OK;
}

// FP64 refresh of C^-1 for the design in P.bits from the FP64 inverse of the
// design bits_ref (a mixed search leaves P.Cinv untouched between refreshes):
// with F the pixels that differ, a block-Woodbury update (eq. lru_woodbury,
// M = |F|) on the matrix cores, exact up to FP64 rounding; a full
// re-inversion when F is larger than kWoodMax or its capacitance matrix is
// singular.  Then E (with one refinement step), R' and x are re-formed.
// defer: the Woodbury status is left for the caller's next wait
// (wood_pending), which must re-invert if it reports a singular update.
int fp64_refresh(pngf_handle* h, bool defer = false, bool tau = false) {
  const int nd = h->pc.n_d;
  pngf::ProbDev& P = h->P;
  h->tau_fresh = false;
  const bool fresh = h->bits_fresh;
  h->bits_fresh = false;
  if (h->opt.precision == PNGF_FP64_PLAIN || h->bits_ref.size() != size_t(nd))
    return device_reinvert(h);
  std::vector<uint8_t> cur(nd);
  if (fresh) {
    cur = h->bits;
  } else {
    HIPCHK(h, hipMemcpyAsync(cur.data(), P.bits, nd, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  std::vector<int32_t> fl;
  for (int i = 0; i < nd; ++i)
    if (cur[i] != h->bits_ref[i]) fl.push_back(i);
  const int k = int(fl.size());
  if (k > pngf::kWoodMax) return device_reinvert(h);
  if (k > 0) {
    bool singular = false;
    int st = woodbury_update(h, fl, cur, &singular, defer);
    if (st) return st;
    if (singular) return device_reinvert(h);
  }
  int st = reform_fields(h, tau);
  if (st) return st;
  h->tau_fresh = tau;
  h->bits_ref = cur;
  h->cinv_stale = false;
  return PNGF_OK;
}

int upload_matrix(pngf_handle* h, z64* dst, const std::vector<cd>& src, int nd) {
  HIPCHK(h, hipMemcpy2DAsync(dst, size_t(h->ld) * sizeof(z64), src.data(), size_t(nd) * sizeof(z64),
                             size_t(nd) * sizeof(z64), nd, hipMemcpyHostToDevice, h->stream));
  return PNGF_OK;
}

int read_state(pngf_handle* h, pngf::DbsState* st) {
  HIPCHK(h, hipMemcpyAsync(st, h->P.st, sizeof(*st), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

int write_state(pngf_handle* h, const pngf::DbsState* st) {
  HIPCHK(h, hipMemcpyAsync(h->P.st, st, sizeof(*st), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

// Stream-ordered write of a state held in pinned memory (no wait: the host
// does not touch it before its next stream-ordered read).
int write_state_pinned(pngf_handle* h, const pngf::DbsState* st) {
  HIPCHK(h, hipMemcpyAsync(h->P.st, st, sizeof(*st), hipMemcpyHostToDevice, h->stream));
  return PNGF_OK;
}


// Ranked search: the keys that step `step` of the segment decides from, under
// a fresh ranking of the state that step reads (buffer set and state of its
// parity): the state's features, the network's scores (or the first-order
// change), then the keys of the best-ranked improving pixels from the exact
// scores the previous step (or the segment start) left, with the cursor back
// at the top of the ranking.  Overwrites the key slots the previous step wrote.
// Stream-ordered, no wait.
int rank_chain(pngf_handle* h, int64_t step) {
  const int nd = h->pc.n_d;
  pngf::ProbDev Q = h->P;
  if (step & 1) {
    for (int f = 0; f < Q.nfreq; ++f) {
      if (Q.CinvB[f]) std::swap(Q.Cinv[f], Q.CinvB[f]);
      std::swap(Q.E[f], Q.EB[f]);
      std::swap(Q.Rp[f], Q.RpB[f]);
      std::swap(Q.tau[f], Q.tauB[f]);
    }
    std::swap(Q.bits, Q.bitsB);
  }
  pngf::DbsState* sin = (step & 1) ? h->P.stB : h->P.st;
  Q.st = sin;   // the features read f and x of the state the next step reads
  const int slot = int(step % 3);
  Timer t(h, KID_OTHER);
  const float* scores = nullptr;
  if (h->rank_model) {
    float* y = nullptr;
    HIPCHK(h, pngf::model_score_state(h->rank_model, Q, &y));
    scores = y;
  } else {
    float* feat = at<float>(h, h->lay.off_feat);
    HIPCHK(h, pngf::launch_features(Q, h->rank_h, h->rank_w, feat, h->stream));
    scores = feat + size_t(kFeatChannels - 1) * nd;
  }
  HIPCHK(h, pngf::launch_ranked_keys(Q, scores, sin, h->opt.precision == PNGF_MIXED ? 1 : 0,
                                     h->P.keys + slot, h->P.keys + 3 + slot, h->stream));
  t.end();
  return PNGF_OK;
}

// Reset the rotating key slots (and, if asked, the panel bookkeeping of the
// state) and score every candidate of the current (normalized) state into
// slot 0; the next step of the search is step 0.  Stream-ordered, no wait.
int start_segment(pngf_handle* h, bool reset_panel = false) {
  HIPCHK(h, pngf::launch_segment_start(h->P, reset_panel ? 1 : 0, h->stream));
  {
    Timer t(h, KID_SCORE);
    HIPCHK(h, pngf::launch_score_rows(h->P, h->npl, nullptr, h->pc.n_d, h->P.keys, h->stream));
    t.end();
  }
  if (h->ranked) return rank_chain(h, 0);
  return PNGF_OK;
}

// start_segment(h, true) right after an FP64 refresh: when that refresh
// formed every candidate's tau beside the fields, the scores come from it
// (k_score_tail, no pass over C^-1 and G).
int start_segment_refreshed(pngf_handle* h) {
  if (!h->tau_fresh) return start_segment(h, true);
  h->tau_fresh = false;
  HIPCHK(h, pngf::launch_segment_start(h->P, 1, h->stream));
  {
    Timer t(h, KID_SCORE);
    HIPCHK(h, pngf::launch_score_tail(h->P, h->P.keys, h->stream));
    t.end();
  }
  if (h->ranked) return rank_chain(h, 0);
  return PNGF_OK;
}

// After an even number of steps the state is back in the A slot; if an odd
// number of updates happened the current vectors/matrix are in the B set:
// swap the roles so that A is current again.
int normalize(pngf_handle* h, pngf::DbsState* st) {
  if (!(st->flips & 1)) return PNGF_OK;
  pngf::ProbDev& P = h->P;
  for (int f = 0; f < P.nfreq; ++f) {
    if (P.CinvB[f]) std::swap(P.Cinv[f], P.CinvB[f]);
    std::swap(P.E[f], P.EB[f]);
    std::swap(P.Rp[f], P.RpB[f]);
    std::swap(P.tau[f], P.tauB[f]);
  }
  std::swap(P.bits, P.bitsB);
  st->flips = 0;
  return write_state_pinned(h, st);
}

// Run `n` (even) steps starting at step index t0, then read the state.
// persist: the n steps of the mixed search as one launch of resident workgroups.
template <class L>
int run_steps(pngf_handle* h, L launch, int64_t t0, int n, pngf::DbsState* pinned,
              bool want_bits = false, bool persist = false) {
  // one event pair around the back-to-back step launches (the average per
  // launch includes the gaps between them)
  Timer t(h, KID_ACCEPT);
  int32_t* pbar = at<int32_t>(h, h->lay.off_pbar);
  if (persist) {
    const hipError_t e = pngf::launch_mixed_persist(
        h->P, int(t0), n, reinterpret_cast<uint64_t*>(pbar), at<int32_t>(h, h->lay.off_flag),
        h->persist_spin, at<double>(h, h->lay.off_band),
        h->wood_pending ? at<int32_t>(h, h->lay.off_status) : nullptr, h->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // refreshes of this search already left the band and a refresh status
      // on the device alone: the per-step kernels cannot take over now
      if (h->persist_ok) return fail(h, PNGF_EDEVICE, "persistent search launch failed");
      // the grid cannot be resident here: one kernel per step from now on
      h->persist_off = true;
      persist = false;
    } else {
      h->persist_ok = true;
    }
  }
  if (!persist)
    for (int b = 0; b < n; ++b) {
      HIPCHK(h, launch(h->P, h->npl, int(t0 + b), h->stream));
      if (h->ranked) {
        const int st = rank_chain(h, t0 + b + 1);
        if (st) return st;
      }
    }
  t.end(n);
  h->bits_fresh = false;
  const int nd = h->pc.n_d;
  // state, time-out flag and (when asked) both design buffers in one copy:
  // they are adjacent in the workspace
  const Layout& Y = h->lay;
  char* stg = h->pin + pngf::kPinStage;
  const size_t span = (want_bits || persist) ? (want_bits ? Y.off_bitsB + nd : Y.off_flag + 4) -
                                                   Y.off_state
                                             : sizeof(pngf::DbsState);
  HIPCHK(h, hipMemcpyAsync(stg, h->ws + Y.off_state, span, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::memcpy(pinned, stg, sizeof(pngf::DbsState));
  const int32_t fl = persist ? *reinterpret_cast<const int32_t*>(stg + (Y.off_flag - Y.off_state))
                             : 0;
  if (persist) h->wood_pending = false;   // the launch read (and acted on) the status
  if (fl == 2) {
    // no step ran: the refresh before it was singular; the caller re-inverts
    HIPCHK(h, hipMemsetAsync(at<int32_t>(h, Y.off_flag), 0, sizeof(int32_t), h->stream));
    h->persist_aborted = true;
    return PNGF_OK;
  }
  if (fl) {
    // the barrier words are left inconsistent: clear them for the next search
    HIPCHK(h, hipMemsetAsync(pbar, 0, pngf::kPersistBarBytes, h->stream));
    HIPCHK(h, hipMemsetAsync(at<int32_t>(h, Y.off_flag), 0, sizeof(int32_t), h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return fail(h, PNGF_ENUMERIC, "a grid barrier of the persistent search timed out");
  }
  if (want_bits) {
    // the design of the last step (in the B set after an odd number of
    // updates); P.bits is one of the two adjacent buffers
    const bool a_first = h->P.bits == at<uint8_t>(h, Y.off_bits);
    const uint8_t* bits_a = reinterpret_cast<const uint8_t*>(stg) +
                            ((a_first ? Y.off_bits : Y.off_bitsB) - Y.off_state);
    const uint8_t* bits_b = reinterpret_cast<const uint8_t*>(stg) +
                            ((a_first ? Y.off_bitsB : Y.off_bits) - Y.off_state);
    const uint8_t* cur = (pinned->flips & 1) ? bits_b : bits_a;
    h->bits.assign(cur, cur + nd);
    h->bits_fresh = true;
  }
  // count only the launches that accepted a flip (the interval also holds
  // the cheap launches that found the search paused or finished)
  if (!h->ev_pool.empty()) {
    const int acc = std::max(0, pinned->n_acc - h->nacc_seen);
    h->ev_pool.back() = reinterpret_cast<hipEvent_t>(intptr_t(KID_ACCEPT) | (intptr_t(acc) << 8));
  }
  h->nacc_seen = pinned->n_acc;
  // (the events are read once, at the end of the search)
  return normalize(h, pinned);
}

// FP64 plain search: one fused step kernel per accepted flip, batches of
// device steps between host checks of the done flag.
int run_plain(pngf_handle* h, pngf::DbsState* pinned) {
  int st = start_segment(h);
  if (st) return st;
  const int batch = 32;
  const int64_t max_steps = int64_t(h->opt.max_accepts) + 2;
  for (int64_t t = 0; t < max_steps + batch; t += batch) {
    st = run_steps(h, pngf::launch_plain_step, t, batch, pinned);
    if (st) return st;
    if (pinned->done) return PNGF_OK;
  }
  return fail(h, PNGF_ENUMERIC, "DBS did not terminate");
}

// At rest P.Cinv is the FP64 inverse of the current design: record that
// design as the base of the block-Woodbury refreshes of a mixed search.
int capture_ref_bits(pngf_handle* h) {
  h->bits_ref.resize(h->pc.n_d);
  HIPCHK(h, hipMemcpyAsync(h->bits_ref.data(), h->P.bits, h->pc.n_d, hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

// While it lives, reform_fields also writes C0^-1 (the complex-FP32 copy)
// from its first pass over C^-1: every path of a mixed refresh ends there.
struct C64Pass {
  pngf_handle* h;
  explicit C64Pass(pngf_handle* hh) : h(hh) { h->reform_c64 = true; }
  ~C64Pass() { h->reform_c64 = false; }
};

// Rescore a refreshed state: segment start (exact FP64 keys), then, with
// `measure`, the FP32 scores' error against them (the band kernel also
// carries a pending block-Woodbury status), else the pending status alone,
// read into the handle's pinned scratch.  Stream-ordered, no wait; the reads
// are valid after the next wait on the bound stream (refresh_settle).
int refresh_rescore(pngf_handle* h, bool measure) {
  const int nd = h->pc.n_d;
  int st = start_segment_refreshed(h);
  if (st) return st;
  double* mo = reinterpret_cast<double*>(h->pin + 8);
  mo[0] = 0.0;
  mo[1] = 0.0;
  int32_t& wst0 = *reinterpret_cast<int32_t*>(h->pin + 24);
  wst0 = 0;
  h->rescore_pending = h->wood_pending;
  double* dband = (h->opt.guard <= 0.0) ? at<double>(h, h->lay.off_band) : nullptr;
  int32_t* dstatus = at<int32_t>(h, h->lay.off_status);
  if (measure) {
    double* out = at<double>(h, h->lay.off_bandout);
    HIPCHK(h, pngf::launch_band_measure(h->P.df32, h->P.dfb, h->P.df, nd, out,
                                        h->rescore_pending ? dstatus : nullptr, h->stream, dband));
    HIPCHK(h, hipMemcpyAsync(mo, out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  } else if (h->rescore_pending) {
    HIPCHK(h, hipMemcpyAsync(&wst0, dstatus, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  }
  return PNGF_OK;
}

// After the wait that follows refresh_rescore: take the measured band, or,
// if the deferred block-Woodbury update turned out singular, re-invert C^-1
// from the design and rescore again (with a wait of its own).
int refresh_settle(pngf_handle* h, bool measure) {
  for (int pass = 0; pass < 2; ++pass) {
    const double* mo = reinterpret_cast<const double*>(h->pin + 8);
    const int32_t wst0 = *reinterpret_cast<const int32_t*>(h->pin + 24);
    const double meas = mo[0];
    const int32_t wst = measure ? int32_t(mo[1]) : wst0;
    const bool pending = h->rescore_pending;
    h->rescore_pending = false;
    h->wood_pending = false;
    if (pending && wst) {
      C64Pass c64pass(h);
      int st = device_reinvert(h);
      if (st) return st;
      st = refresh_rescore(h, measure);
      if (st) return st;
      if (measure) HIPCHK(h, hipStreamSynchronize(h->stream));
      continue;
    }
    if (measure && std::isfinite(meas) && h->opt.guard <= 0.0)
      h->P.band = std::min(1e-2, std::max(1e-6, 100.0 * meas));
    return PNGF_OK;
  }
  return PNGF_OK;
}

// Re-form the FP64 state, cast C0^-1 to complex FP32, rescore every candidate
// in FP64 (exact key) and, when the previous scores were FP32, measure their
// error against the FP64 scores to set the error band.
// nosync (persistent search): nothing is read back; the band goes to the
// device word only and a pending block-Woodbury status is checked by the
// next launch (which runs no step if it is set).
int mixed_refresh(pngf_handle* h, bool measure, bool nosync = false) {
  const int nd = h->pc.n_d;
  h->wood_pending = false;
  int st;
  {
    C64Pass c64pass(h);
    st = fp64_refresh(h, true, true);
  }
  if (st) return st;
  if (nosync) {
    double* dband = (h->opt.guard <= 0.0) ? at<double>(h, h->lay.off_band) : nullptr;
    st = start_segment_refreshed(h);
    if (st) return st;
    if (measure && dband)
      HIPCHK(h, pngf::launch_band_measure(h->P.df32, h->P.dfb, h->P.df, nd,
                                          at<double>(h, h->lay.off_bandout), nullptr, h->stream,
                                          dband));
    return PNGF_OK;
  }
  st = refresh_rescore(h, measure);
  if (st) return st;
  if (measure || h->rescore_pending) HIPCHK(h, hipStreamSynchronize(h->stream));
  return refresh_settle(h, measure);
}

// FP64 residual |b - C E| / |b| of frequency 0 (drift monitor).
int mixed_residual(pngf_handle* h, double* ratio) {
  const int nd = h->pc.n_d;
  const Layout& L = h->lay;
  pngf::ProbDev& P = h->P;
  z64* r = at<z64>(h, L.off_r[0]);
  const z64* b = at<z64>(h, L.off_b[0]);
  HIPCHK(h, pngf::launch_gemv(P.G[0], h->ld, nd, P.E[0], P.bits, P.deps, z64{P.k0sq[0], 0.0},
                              z64{1.0, 0.0}, b, -1.0, P.E[0], r, h->stream));
  std::vector<z64> rh(nd), bh(nd);
  HIPCHK(h, hipMemcpyAsync(rh.data(), r, nd * sizeof(z64), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(bh.data(), b, nd * sizeof(z64), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  double nr = 0.0, nb = 0.0;
  for (int i = 0; i < nd; ++i) {
    nr += rh[i].re * rh[i].re + rh[i].im * rh[i].im;
    nb += bh[i].re * bh[i].re + bh[i].im * bh[i].im;
  }
  *ratio = std::sqrt(nr / std::max(nb, 1e-300));
  return PNGF_OK;
}

// The periodic refresh of the persistent mixed search, queued right behind
// the batch of steps it follows, before the host has read that batch's end
// state: the parity fix of the buffers, the flip list, its scales and the
// measurement gate come from the device (k_wood_prep, which also records the
// design C^-1 will hold and starts the next segment: state bookkeeping and
// key slots); the block-Woodbury update runs on kpad = k_refresh
// columns (padding entries: pixel 0 with scale 0, which leave the result
// unchanged); then the field re-formation (which also writes C0^-1), the FP64
// rescoring and, when the scores were FP32, the band measurement.  If the
// batch ended the search, this re-forms the final design's state (which the
// final refresh then finds done); a singular capacitance matrix or more
// flips than kpad leave the status word set, and the next batch runs no step.
int refresh_ahead(pngf_handle* h) {
  const int nd = h->pc.n_d, ld = h->ld;
  const Layout& L = h->lay;
  pngf::ProbDev& P = h->P;
  const int kpad = h->opt.k_refresh;
  int32_t* dF = at<int32_t>(h, L.off_wF);
  double* dS = at<double>(h, L.off_wS);
  int32_t* wk = at<int32_t>(h, L.off_wk);
  int32_t* status = at<int32_t>(h, L.off_status);
  uint8_t* bref = at<uint8_t>(h, L.off_bref);
  const z64 one{1.0, 0.0}, zero{0.0, 0.0};
  HIPCHK(h, pngf::launch_wood_prep(P, bref, kpad, dF, dS, wk, h->stream));
  {
    Timer t(h, KID_WOOD);
    z64* wP = at<z64>(h, L.off_wP[0]);
    z64* wW = at<z64>(h, L.off_wW[0]);
    z64* cap = at<z64>(h, L.off_wCap[0]);
    z64* work = at<z64>(h, L.off_wWork[0]);
    int nzp = 0;
    HIPCHK(h, pngf::launch_zgemm(nd, kpad, nd, P.Cinv[0], ld, nullptr, P.G[0], ld, true, dF, wP,
                                 kpad, one, zero, pngf::kWoodSplits, work, h->stream, &nzp));
    if (nzp > 0)
      HIPCHK(h, pngf::launch_wood_panel(work, nzp, nd, kpad, dS, wP, kpad, dF, cap, status,
                                        h->stream, wk));
    else
      HIPCHK(h, pngf::launch_wood_cap(wP, kpad, nd, dF, kpad, dS, cap, status, h->stream, wk));
    HIPCHK(h, pngf::launch_small_inverse(cap, kpad, status, h->stream));
    if (h->force_singular > 0) {
      // test hook: this refresh reports a singular capacitance matrix
      HIPCHK(h, hipMemsetAsync(status, 1, sizeof(int32_t), h->stream));
      --h->force_singular;
    }
    HIPCHK(h, pngf::launch_zgemm(kpad, nd, kpad, cap, kpad, nullptr, P.Cinv[0], ld, false, dF,
                                 wW, nd, one, zero, 1, nullptr, h->stream));
    HIPCHK(h, pngf::launch_zgemm(nd, nd, kpad, wP, kpad, nullptr, wW, nd, false, nullptr,
                                 P.Cinv[0], ld, one, one, 1, nullptr, h->stream));
    t.end(1);
  }
  int st;
  {
    C64Pass c64pass(h);
    st = reform_fields(h, true, false);   // with every candidate's tau, x left to the tail
  }
  if (st) return st;
  {
    // x and f, every candidate's score and key (the segment's start was done
    // by k_wood_prep), and the band measurement when the scores were FP32
    Timer t(h, KID_SCORE);
    const cd xb = h->pc.freq[0].xb;
    const bool band = h->opt.guard <= 0.0;
    HIPCHK(h, pngf::launch_refresh_tail(P, at<z64>(h, L.off_god[0]), z64{xb.real(), xb.imag()},
                                        P.keys, P.df32, P.dfb,
                                        band ? at<double>(h, L.off_bandout) : nullptr,
                                        band ? at<double>(h, L.off_band) : nullptr, wk + 1,
                                        h->stream));
    t.end();
  }
  h->bits_fresh = false;
  return PNGF_OK;
}

// The periodic persistent mixed search with each refresh queued ahead of the
// host (refresh_ahead): per round, a batch that runs until the search asks
// for its refresh (k_refresh accepts, a band hit) or ends, the read of its
// end state, then the refresh; the host waits for the state read only, so
// it queues the next batch while the refresh runs.  On return `pinned`
// holds the final state, its FP64 fields re-formed.  Returns 1 (nothing
// done) if the grid of the persistent search cannot be resident here.
int run_mixed_ahead(pngf_handle* h, pngf::DbsState* pinned, int64_t* n_refresh, int64_t* n_band) {
  const int nd = h->pc.n_d;
  const Layout& Y = h->lay;
  int32_t* status = at<int32_t>(h, Y.off_status);
  int32_t* pbar = at<int32_t>(h, Y.off_pbar);
  uint8_t* bref = at<uint8_t>(h, Y.off_bref);
  char* stg = h->pin + pngf::kPinStage;
  const size_t span = Y.off_flag + 4 - Y.off_state;
  // a batch asks for its refresh at the decision after k_refresh accepts
  const int nl = (h->opt.k_refresh + 2) & ~1;
  HIPCHK(h, hipMemcpyAsync(bref, h->P.bits, nd, hipMemcpyDeviceToDevice, h->stream));
  bool after_refresh = false;   // a refresh is queued before this batch
  const int64_t max_rounds = 4 * int64_t(h->opt.max_accepts) + 64;
  for (int64_t round = 0; round < max_rounds; ++round) {
    size_t tag = size_t(-1);   // the batch's entry in the event pool, if timed
    {
      Timer t(h, KID_ACCEPT);
      const hipError_t e = pngf::launch_mixed_persist(
          h->P, 0, nl, reinterpret_cast<uint64_t*>(pbar), at<int32_t>(h, Y.off_flag),
          h->persist_spin, at<double>(h, Y.off_band), after_refresh ? status : nullptr,
          h->stream);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        if (h->persist_ok || round > 0) return fail(h, PNGF_EDEVICE, "persistent search launch failed");
        h->persist_off = true;
        return 1;
      }
      h->persist_ok = true;
      t.end(nl);
      if (t.a) tag = h->ev_pool.size() - 1;
    }
    HIPCHK(h, hipMemcpyAsync(stg, h->ws + Y.off_state, span, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipEventRecord(h->ev_ahead, h->stream));
    int st = refresh_ahead(h);
    if (st) return st;
    after_refresh = true;
    HIPCHK(h, hipEventSynchronize(h->ev_ahead));
    std::memcpy(pinned, stg, sizeof(pngf::DbsState));
    const int32_t fl = *reinterpret_cast<const int32_t*>(stg + (Y.off_flag - Y.off_state));
    if (tag != size_t(-1)) {
      // count only the accepted flips of the batch
      const int acc = std::max(0, pinned->n_acc - h->nacc_seen);
      h->ev_pool[tag] = reinterpret_cast<hipEvent_t>(intptr_t(KID_ACCEPT) | (intptr_t(acc) << 8));
    }
    h->nacc_seen = pinned->n_acc;
    if (fl == 2) {
      // no step ran: the refresh before this batch was singular (or had more
      // flips than it holds); the one queued behind it started from an
      // unusable C^-1 too: re-invert from the design
      HIPCHK(h, hipStreamSynchronize(h->stream));
      HIPCHK(h, hipMemsetAsync(at<int32_t>(h, Y.off_flag), 0, sizeof(int32_t), h->stream));
      h->reform_c64 = true;
      st = device_reinvert(h);
      h->reform_c64 = false;
      if (st) return st;
      HIPCHK(h, hipMemcpyAsync(bref, h->P.bits, nd, hipMemcpyDeviceToDevice, h->stream));
      st = start_segment(h, true);
      if (st) return st;
      after_refresh = false;
      continue;
    }
    if (fl) {
      HIPCHK(h, hipStreamSynchronize(h->stream));
      HIPCHK(h, hipMemsetAsync(pbar, 0, pngf::kPersistBarBytes, h->stream));
      HIPCHK(h, hipMemsetAsync(at<int32_t>(h, Y.off_flag), 0, sizeof(int32_t), h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      return fail(h, PNGF_ENUMERIC, "a grid barrier of the persistent search timed out");
    }
    if (pinned->done) {
      // the refresh queued behind the last batch re-formed the FP64 state of
      // the final design (what the final refresh of a search computes), unless
      // its update failed: then re-invert.  The final state comes with the
      // same wait.
      int32_t& sth = *reinterpret_cast<int32_t*>(h->pin + 24);
      sth = 0;
      HIPCHK(h, hipMemcpyAsync(&sth, status, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipMemcpyAsync(stg, bref, nd, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipMemcpyAsync(pinned, h->P.st, sizeof(pngf::DbsState), hipMemcpyDeviceToHost,
                               h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      h->bits_ref.assign(reinterpret_cast<const uint8_t*>(stg),
                         reinterpret_cast<const uint8_t*>(stg) + nd);
      if (sth) {
        st = device_reinvert(h);
        if (st) return st;
        HIPCHK(h, hipMemcpyAsync(pinned, h->P.st, sizeof(pngf::DbsState),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
      }
      return PNGF_OK;
    }
    *n_refresh += 1;
    if (pinned->need_refresh == 2) *n_band += 1;
  }
  return fail(h, PNGF_ENUMERIC, "DBS did not terminate");
}

// Mixed search: complex-FP32 steps in batches; between batches the host
// re-inverts in FP64 when the device asks (interval, full panel, a band hit),
// folds the panel into C0^-1 on the matrix cores, or checks the drift.
int run_mixed(pngf_handle* h, pngf::DbsState* pinned, int64_t* n_refresh, int64_t* n_band) {
  const int nd = h->pc.n_d, F = int(h->pc.freq.size());
  // the state's mixed bookkeeping was reset by the search prologue
  for (int f = 0; f < F; ++f)
    HIPCHK(h, pngf::launch_to_c64(h->P.Cinv[f], h->P.C0[f], nd, h->ld, h->stream));
  int st = start_segment(h);
  if (st) return st;
  // a periodic persistent search queues each refresh ahead of the host (the
  // design C^-1 holds is kept on the device); otherwise the host keeps it
  const bool ahead = !h->persist_off && !h->ranked && F == 1 && nd <= 2048 &&
                     h->P.kcap <= pngf::kPersistSlotsHost &&
                     !(h->opt.flags & PNGF_FLAG_STEP_LAUNCHES) && h->opt.k_refresh > 0 &&
                     h->opt.k_refresh <= pngf::kAheadMaxK &&
                     (h->opt.k_fold == 0 || h->opt.k_fold >= h->opt.k_refresh);
  if (!ahead) {
    st = capture_ref_bits(h);
    if (st) return st;
  }
  if (ahead) {
    st = run_mixed_ahead(h, pinned, n_refresh, n_band);
    if (st == 1) {
      st = capture_ref_bits(h);
      if (st) return st;
    } else {
      return st;
    }
    // the persistent grid cannot be resident: one launch per step below
  }
  const int64_t max_rounds = 4 * int64_t(h->opt.max_accepts) + 64;
  int64_t t = 0;                 // step index within the segment
  int64_t since = 0, kpan = 0;   // host view of n_since / kpanel
  int64_t checked = 0;           // n_since at the last drift check
  for (int64_t round = 0; round < max_rounds; ++round) {
    const bool persist = !h->persist_off && !h->ranked && F == 1 && nd <= 2048 &&
                         h->P.kcap <= pngf::kPersistSlotsHost &&
                         !(h->opt.flags & PNGF_FLAG_STEP_LAUNCHES);
    // end the batch where a periodic re-inversion or a fold is due, so that
    // few launches of the batch find the search paused; batches stay even.
    // Persistent batches of a periodic search run a whole refresh period
    // (the host has nothing to check in between).
    int nb = (persist && h->opt.k_refresh > 0) ? pngf::kPersistBatch : pngf::kMixedBatch;
    if (h->opt.k_refresh > 0) nb = int(std::min<int64_t>(nb, std::max<int64_t>(1, h->opt.k_refresh - since)));
    if (h->opt.k_fold > 0) nb = int(std::min<int64_t>(nb, std::max<int64_t>(1, h->opt.k_fold - kpan)));
    nb += nb & 1;
    // read the design with the batch when it ends at a periodic refresh
    const bool due = h->opt.k_refresh > 0 && since + nb >= h->opt.k_refresh;
    // a persistent batch that ends at a periodic refresh runs on to the
    // decision that asks for it (one host round trip less)
    const int nl = (persist && due) ? nb + 2 : nb;
    st = run_steps(h, pngf::launch_mixed_step, t, nl, pinned, due, persist);
    if (st) return st;
    if (h->persist_aborted) {
      // the unchecked block-Woodbury refresh before this batch was singular
      // and the batch ran no step: re-invert and run it again
      h->persist_aborted = false;
      h->reform_c64 = true;
      st = device_reinvert(h);
      h->reform_c64 = false;
      if (st) return st;
      st = start_segment(h, true);
      if (st) return st;
      continue;
    }
    t += nl;
    if (pinned->done) break;
    bool refresh = pinned->need_refresh != 0;
    const bool band_hit = pinned->need_refresh == 2;
    if (!refresh && h->opt.k_refresh == 0 && !pinned->exact &&
        pinned->n_since >= checked + pngf::kDriftEvery) {
      checked = pinned->n_since;
      double ratio = 0.0;
      st = mixed_residual(h, &ratio);
      if (st) return st;
      refresh = ratio > pngf::kDriftTol;
    }
    since = pinned->n_since;
    kpan = pinned->kpanel;
    if (refresh) {
      // with the persistent search running, the refresh reads nothing back
      st = mixed_refresh(h, !pinned->exact, persist && h->persist_ok && !h->persist_off);
      if (st) return st;
      *n_refresh += 1;
      if (band_hit) *n_band += 1;
      since = kpan = checked = 0;
      t = 0;
    } else if (pinned->kpanel >= pngf::kPanelCap - pngf::kMixedBatch ||
               (h->opt.k_fold > 0 && pinned->kpanel >= h->opt.k_fold)) {
      Timer tm(h, KID_FOLD);
      for (int f = 0; f < F; ++f) {
        HIPCHK(h, pngf::launch_fold_q(h->P, f, pinned->kpanel, h->stream));
        HIPCHK(h, pngf::launch_fold(h->P, f, pinned->kpanel, h->stream));
      }
      tm.end();
      pngf::DbsState s2;
      st = read_state(h, &s2);
      if (st) return st;
      s2.kpanel = 0;
      st = write_state(h, &s2);
      if (st) return st;
      kpan = 0;
    }
  }
  if (!pinned->done) return fail(h, PNGF_ENUMERIC, "DBS did not terminate");
  // Final objective in FP64: re-form the state of the converged design.
  st = fp64_refresh(h);
  if (st) return st;
  HIPCHK(h, hipMemcpyAsync(pinned, h->P.st, sizeof(pngf::DbsState), hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}


// An R-form search leaves C^-1 at the design of its start: bring it to the
// current design (block Woodbury, or a re-inversion) before a call needs it.
int ensure_cinv(pngf_handle* h) {
  if (!h->cinv_stale) return PNGF_OK;
  return fp64_refresh(h);
}

// T0 = C^-1 G for the current design: rows of G for pixels at eps_lo, then
// T0 += C^-1[:,S] G[S,:] over the pixels S at eps_hi (identity columns of
// C^-1 elsewhere), on the FP64 matrix cores.
int build_t0(pngf_handle* h) {
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  pngf::ProbDev& P = h->P;
  std::vector<int32_t> sidx;
  for (int i = 0; i < nd; ++i)
    if (h->bits_ref[i]) sidx.push_back(i);
  const int ns = int(sidx.size());
  int32_t* d_sidx = at<int32_t>(h, h->lay.off_sidx);
  if (ns > 0)
    HIPCHK(h, hipMemcpyAsync(d_sidx, sidx.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice,
                             h->stream));
  for (int f = 0; f < F; ++f) {
    Timer t(h, KID_LU);
    HIPCHK(h, pngf::launch_rform_t0_init(P, f, h->stream));
    if (ns > 0)
      HIPCHK(h, pngf::launch_zgemm(nd, nd, ns, P.Cinv[f], ld, d_sidx, P.G[f], ld, false, d_sidx,
                                   P.T0[f], ld, z64{1.0, 0.0}, z64{1.0, 0.0}, 1, nullptr,
                                   h->stream));
    t.end();
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));   // sidx (host) was read by the copy
  return PNGF_OK;
}

// Fold the R-form panel into T0 (T0 += Ut U) and empty it.
int rform_fold(pngf_handle* h, int kp) {
  const int nd = h->pc.n_d, ld = h->ld, F = int(h->pc.freq.size());
  pngf::ProbDev& P = h->P;
  z64* Ut = at<z64>(h, h->lay.off_Ut);
  for (int f = 0; f < F; ++f) {
    Timer t(h, KID_FOLD);
    HIPCHK(h, pngf::launch_rform_ut(P, f, kp, Ut, h->stream));
    HIPCHK(h, pngf::launch_zgemm(nd, nd, kp, Ut, kp, nullptr, P.Up[f], ld, false, nullptr,
                                 P.T0[f], ld, z64{1.0, 0.0}, z64{1.0, 0.0}, 1, nullptr,
                                 h->stream));
    t.end();
  }
  return PNGF_OK;
}

// R-form search (FP64, exact): T0 once, then one O(N_d k) step kernel per
// accepted flip; the panel is folded into T0 when it is full, and with
// k_refresh > 0 the whole state is re-anchored on an FP64 C^-1 every
// k_refresh accepts.
int run_rform(pngf_handle* h, pngf::DbsState* pinned) {
  int st = ensure_cinv(h);
  if (st) return st;
  st = capture_ref_bits(h);
  if (st) return st;
  st = build_t0(h);
  if (st) return st;
  pngf::DbsState s;
  st = read_state(h, &s);
  if (st) return st;
  s.kpanel = 0;
  s.n_since = 0;
  s.exact = 1;
  s.need_refresh = 0;
  s.flips = 0;
  st = write_state(h, &s);
  if (st) return st;
  st = start_segment(h);   // tau of the start state (from C^-1) and the first keys
  if (st) return st;
  h->cinv_stale = true;
  const int batch = 64;   // steps are cheap: fewer host checks
  const int64_t max_rounds = 4 * int64_t(h->opt.max_accepts) + 64;
  int64_t t = 0;
  for (int64_t round = 0; round < max_rounds; ++round) {
    st = run_steps(h, pngf::launch_rform_step, t, batch, pinned);
    if (st) return st;
    t += batch;
    if (pinned->done) return PNGF_OK;
    if (pinned->need_refresh && h->P.k_refresh > 0 && pinned->n_since >= h->P.k_refresh) {
      // re-anchor: C^-1 for the current design by a full FP64 re-inversion,
      // E, R' and x re-formed from it, T0 rebuilt, every candidate rescored
      // from C^-1 (the panel's rank-1 terms are dropped).  Not a block-
      // Woodbury update of the previous anchor's C^-1: T0 = C^-1 G inherits
      // C^-1's error directly, and chained Woodbury updates through an
      // ill-conditioned capacitance matrix (conducting pixels) leave C^-1
      // at ~1e-10 instead of ~1e-13.
      st = device_reinvert(h);
      if (st) return st;
      st = capture_ref_bits(h);
      if (st) return st;
      st = build_t0(h);
      if (st) return st;
      h->cinv_stale = true;
      st = read_state(h, pinned);
      if (st) return st;
      pinned->kpanel = 0;
      pinned->n_since = 0;
      pinned->need_refresh = 0;
      pinned->exact = 1;
      st = write_state(h, pinned);
      if (st) return st;
      st = start_segment(h);
      if (st) return st;
      t = 0;
    } else if (pinned->need_refresh) {
      st = rform_fold(h, pinned->kpanel);
      if (st) return st;
      pinned->kpanel = 0;
      pinned->need_refresh = 0;
      pinned->exact = 1;
      st = write_state(h, pinned);
      if (st) return st;
      const uint32_t none[6] = {pngf::kNoKey, pngf::kNoKey, pngf::kNoKey,
                                pngf::kNoKey, pngf::kNoKey, pngf::kNoKey};
      HIPCHK(h, hipMemcpyAsync(h->P.keys, none, sizeof(none), hipMemcpyHostToDevice, h->stream));
      HIPCHK(h, pngf::launch_rform_score(h->P, h->stream));
      if (h->ranked) {
        st = rank_chain(h, 0);
        if (st) return st;
      }
      HIPCHK(h, hipStreamSynchronize(h->stream));
      t = 0;
    }
  }
  return fail(h, PNGF_ENUMERIC, "DBS did not terminate");
}


// Validate and upload the sweep orders and reset the search bookkeeping of a
// bound handle with a design (queued, no wait; the state records the initial
// objective as f_start).  The design's initial inverse is checked by the
// caller, after this is queued.
int dbs_prologue(pngf_handle* h, const int32_t* perms, int32_t n_sweeps) {
  int st = check_ready(h, true, false);
  if (st) return st;
  const int nd = h->pc.n_d;
  if (!perms || n_sweeps < 1 || n_sweeps > h->opt.max_sweeps)
    return fail(h, PNGF_EINVAL, "n_sweeps must be in [1, max_sweeps]");
  std::vector<int32_t> rank(size_t(n_sweeps) * nd, -1);
  for (int s = 0; s < n_sweeps; ++s)
    for (int q = 0; q < nd; ++q) {
      const int32_t m = perms[size_t(s) * nd + q];
      if (m < 0 || m >= nd || rank[size_t(s) * nd + m] != -1)
        return fail(h, PNGF_EINVAL, "perms must hold permutations of the pixel ids");
      rank[size_t(s) * nd + m] = q;
    }
  // the visiting orders and their ranks go up from the pinned staging area
  // when they fit behind the state (read back into only after these copies,
  // on the same stream), else from the caller's memory
  const size_t pb = rank.size() * sizeof(int32_t);
  char* stg = h->pin + pngf::kPinStage;
  const bool staged = pngf::kStageOrders + 2 * pb <= h->pin_idx - pngf::kPinStage;
  const void* src_p = perms;
  const void* src_r = rank.data();
  if (staged) {
    std::memcpy(stg + pngf::kStageOrders, perms, pb);
    std::memcpy(stg + pngf::kStageOrders + pb, rank.data(), pb);
    src_p = stg + pngf::kStageOrders;
    src_r = stg + pngf::kStageOrders + pb;
  }
  HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(h->P.perm), src_p, pb, hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(h->P.rank), src_r, pb, hipMemcpyHostToDevice,
                           h->stream));
  // every search starts from the initial error band (it is recalibrated at
  // each FP64 re-inversion), so repeated runs are identical
  h->P.band = (h->opt.guard > 0.0) ? h->opt.guard : 1e-3;
  // from pinned memory (a copy from pageable memory can wait for the stream)
  auto* pband = reinterpret_cast<double*>(h->pin + pngf::kPinBand);
  *pband = h->P.band;
  HIPCHK(h, hipMemcpyAsync(at<double>(h, h->lay.off_band), pband, sizeof(double),
                           hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < KID_N; ++k) { h->ktime_ms[k] = 0.0; h->klaunch[k] = 0; }
  h->nacc_seen = 0;
  h->persist_ok = false;
  h->persist_aborted = false;
  // the state's bookkeeping reset on the device (its objective, from the
  // fields of the current design, becomes the search's starting value): no
  // round trip
  HIPCHK(h, pngf::launch_state_begin(h->P.st, n_sweeps, h->opt.eta, h->stream));
  return PNGF_OK;
}

// Copy the accept log and fill the result summary.
int dbs_epilogue(pngf_handle* h, const pngf::DbsState& fin, int64_t n_refresh, int64_t n_band,
                 int32_t* accepted, double* f_trace, pngf_dbs_result* res) {
  const int nd = h->pc.n_d;
  const int na = fin.n_acc;
  // logs and design through the pinned staging area: three copies, one wait
  const size_t lpb = (size_t(na) * sizeof(int32_t) + 7) & ~size_t(7);
  char* stg = h->pin + pngf::kPinStage;
  if (lpb + size_t(na) * sizeof(double) + nd > h->pin_idx - pngf::kPinStage)
    return fail(h, PNGF_EINVAL, "more accepts than the handle's max_accepts");
  auto* lp = reinterpret_cast<int32_t*>(stg);
  auto* lf = reinterpret_cast<double*>(stg + lpb);
  auto* lb = reinterpret_cast<uint8_t*>(lf + na);
  if (accepted && na > 0)
    HIPCHK(h, hipMemcpyAsync(lp, h->P.log_pix, na * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  if (f_trace && na > 0)
    HIPCHK(h, hipMemcpyAsync(lf, h->P.log_f, na * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(lb, h->P.bits, nd, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (accepted && na > 0) std::memcpy(accepted, lp, na * sizeof(int32_t));
  if (f_trace && na > 0) std::memcpy(f_trace, lf, na * sizeof(double));
  std::memcpy(h->bits.data(), lb, nd);
  if (h->opt.flags & (PNGF_FLAG_TIMING | PNGF_FLAG_TIMING_STEPS)) collect_times(h);
  if (!std::isfinite(fin.f)) return fail(h, PNGF_ENUMERIC, "objective is not finite");
  if (res) {
    res->n_accepted = na;
    res->sweeps = fin.sweeps;
    res->converged = fin.converged;
    res->n_refresh = int32_t(n_refresh);
    res->attempts = fin.attempts;
    res->n_verified = n_band;
    res->f_initial = fin.f_start;
    res->f_final = fin.f;
  }
  h->f_host = fin.f;
  return PNGF_OK;
}

}  // namespace

extern "C" {

const char* pngf_version(void) { return "pngf 0.1 (gfx950)"; }

const char* pngf_last_error(const pngf_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

int pngf_precompute(const pngf_problem* p, pngf_handle** out) {
  if (!out) return fail(nullptr, PNGF_EINVAL, "null output pointer");
  *out = nullptr;
  if (p && p->nfreq > pngf::kMaxFreq)
    return fail(nullptr, PNGF_EINVAL, "at most 8 frequencies per handle");
  pngf_handle* h = new (std::nothrow) pngf_handle();
  if (!h) return fail(nullptr, PNGF_ENOMEM, "out of host memory");
  std::string err;
  int st;
  try {
    st = pngf::precompute(p, &h->pc, &err);
  } catch (const std::bad_alloc&) {
    st = PNGF_ENOMEM;
    err = "out of host memory in precompute";
  }
  if (st != PNGF_OK) {
    delete h;
    return fail(nullptr, st, err);
  }
  h->ld = ((h->pc.n_d + 63) / 64) * 64;
  h->npl = npl_for(h->pc.n_d);
  h->bits.assign(h->pc.n_d, 0);
  *out = h;
  return PNGF_OK;
}

int pngf_sizes(pngf_handle* h, int32_t* n_d, int32_t* nfreq) {
  if (!h) return PNGF_EINVAL;
  if (n_d) *n_d = h->pc.n_d;
  if (nfreq) *nfreq = int32_t(h->pc.freq.size());
  return PNGF_OK;
}

int pngf_precompute_seconds(pngf_handle* h, double* s) {
  if (!h || !s) return PNGF_EINVAL;
  *s = h->pc.seconds;
  return PNGF_OK;
}

int pngf_get_precompute(pngf_handle* h, int32_t fi, double* G, double* b, double* god,
                        double* xb) {
  if (!h) return PNGF_EINVAL;
  if (fi < 0 || fi >= int(h->pc.freq.size())) return fail(h, PNGF_EINVAL, "frequency index out of range");
  const pngf::FreqData& F = h->pc.freq[fi];
  const size_t nd = h->pc.n_d;
  if (G) std::memcpy(G, F.G.data(), nd * nd * sizeof(cd));
  if (b) std::memcpy(b, F.b.data(), nd * sizeof(cd));
  if (god) std::memcpy(god, F.god.data(), nd * sizeof(cd));
  if (xb) std::memcpy(xb, &F.xb, sizeof(cd));
  return PNGF_OK;
}

int pngf_objective_norm(pngf_handle* h, int32_t fi, double* norm) {
  if (!h || !norm) return PNGF_EINVAL;
  if (fi < 0 || fi >= int(h->pc.freq.size())) return fail(h, PNGF_EINVAL, "frequency index out of range");
  *norm = h->pc.freq[fi].norm;
  return PNGF_OK;
}

int pngf_workspace_bytes(pngf_handle* h, const pngf_options* o, size_t* bytes) {
  if (!h || !o || !bytes) return PNGF_EINVAL;
  if (o->precision != PNGF_FP64_PLAIN && o->precision != PNGF_MIXED && o->precision != PNGF_RFORM)
    return fail(h, PNGF_EINVAL, "precision must be PNGF_FP64_PLAIN, PNGF_MIXED or PNGF_RFORM");
  if (o->max_tile < 0 || o->max_tile > pngf::kWoodMax)
    return fail(h, PNGF_EINVAL, "max_tile must be in [0, 64]");
  *bytes = make_layout(h, o).total;
  return PNGF_OK;
}

int pngf_bind(pngf_handle* h, const pngf_options* o, void* dev_ws, size_t bytes, void* stream) {
  if (!h || !o || !dev_ws) return PNGF_EINVAL;
  if (o->precision != PNGF_FP64_PLAIN && o->precision != PNGF_MIXED && o->precision != PNGF_RFORM)
    return fail(h, PNGF_EINVAL, "precision must be PNGF_FP64_PLAIN, PNGF_MIXED or PNGF_RFORM");
  if (o->k_refresh < 0 || o->k_fold < 0) return fail(h, PNGF_EINVAL, "k_refresh and k_fold must be >= 0");
  if (o->max_accepts < 1 || o->max_sweeps < 1)
    return fail(h, PNGF_EINVAL, "max_accepts and max_sweeps must be >= 1");
  if (o->max_tile < 0 || o->max_tile > pngf::kWoodMax ||
      (o->max_tile > 0 && o->precision != PNGF_FP64_PLAIN))
    return fail(h, PNGF_EINVAL, "max_tile must be in [0, 64], and 0 unless PNGF_FP64_PLAIN");
  if (h->pc.n_d > pngf::kMaxPixels) return fail(h, PNGF_EINVAL, "at most 16384 design pixels");
  if (reinterpret_cast<uintptr_t>(dev_ws) & 255)
    return fail(h, PNGF_EINVAL, "workspace must be 256-byte aligned");
  Layout L = make_layout(h, o);
  if (bytes < L.total) return fail(h, PNGF_ENOMEM, "workspace too small");
  if (h->inv_pending) {
    // an initial inverse still queued on the old binding: let it finish (its
    // result is dropped with the design)
    HIPCHK(h, hipEventSynchronize(h->ev_inv));
    h->inv_pending = false;
  }
  h->opt = *o;
  h->lay = L;
  h->bits_fresh = false;
  h->wood_pending = false;
  h->ws = static_cast<char*>(dev_ws);
  h->ws_bytes = bytes;
  h->stream = static_cast<hipStream_t>(stream);
  const int nd = h->pc.n_d, F = int(h->pc.freq.size());
  if (int(h->aux.size()) != F - 1) {
    release_streams(h);
    for (int f = 1; f < F; ++f) {
      hipStream_t a = nullptr;
      hipEvent_t e = nullptr;
      HIPCHK(h, hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
      h->aux.push_back(a);
      HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      h->ev_join.push_back(e);
    }
    if (F > 1) HIPCHK(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
  }
  pngf::ProbDev& P = h->P;
  P = pngf::ProbDev{};
  P.nd = nd;
  P.ld = h->ld;
  P.nfreq = F;
  P.max_acc = o->max_accepts;
  // PEC pixels: the transposed j-form is a field-form system with G - I in
  // place of G and kappa = -1 in place of k0^2 deps (eq. currequiv_j_disc).
  const bool pec = h->pc.pec;
  P.deps = pec ? -1.0 : h->pc.eps_hi - h->pc.eps_lo;
  for (int f = 0; f < F; ++f) {
    P.k0sq[f] = pec ? 1.0 : h->pc.freq[f].k0 * h->pc.freq[f].k0;
    P.coef[f] = 1.0 / (F * h->pc.freq[f].norm);
    P.G[f] = at<z64>(h, L.off_G[f]);
    P.Cinv[f] = at<z64>(h, L.off_C[f]);
    P.E[f] = at<z64>(h, L.off_E[f]);
    P.Rp[f] = at<z64>(h, L.off_Rp[f]);
    P.tau[f] = at<z64>(h, L.off_tau[f]);
    P.q[f] = at<z64>(h, L.off_q[f]);
  }
  P.bits = at<uint8_t>(h, L.off_bits);
  P.perm = at<int32_t>(h, L.off_perm);
  P.rank = at<int32_t>(h, L.off_rank);
  P.log_pix = at<int32_t>(h, L.off_logp);
  P.log_f = at<double>(h, L.off_logf);
  P.df = at<double>(h, L.off_df);
  P.st = at<pngf::DbsState>(h, L.off_state);
  for (int f = 0; f < F; ++f) {
    P.CinvB[f] = (o->precision == PNGF_FP64_PLAIN) ? at<z64>(h, L.off_CB[f]) : nullptr;
    P.EB[f] = at<z64>(h, L.off_EB[f]);
    P.RpB[f] = at<z64>(h, L.off_RpB[f]);
    P.tauB[f] = at<z64>(h, L.off_tauB[f]);
  }
  P.bitsB = at<uint8_t>(h, L.off_bitsB);
  P.stB = at<pngf::DbsState>(h, L.off_stateB);
  P.keys = at<uint32_t>(h, L.off_keys);
  P.pm = at<int32_t>(h, L.off_pm);
  P.kcap = pngf::kPanelCap;
  P.k_refresh = o->k_refresh;
  P.band = (o->guard > 0.0) ? o->guard : 1e-3;
  if (o->precision == PNGF_MIXED) {
    for (int f = 0; f < F; ++f) {
      P.C0[f] = at<z32>(h, L.off_C0[f]);
      P.G32[f] = at<z32>(h, L.off_G32[f]);
      P.Pp[f] = at<z32>(h, L.off_Pp[f]);
      P.Qp[f] = at<z32>(h, L.off_Qp[f]);
      P.alph[f] = at<z64>(h, L.off_alph[f]);
      P.pcoef[f] = at<z64>(h, L.off_pcoef[f]);
    }
    P.df32 = at<double>(h, L.off_df32);
    P.dfb = at<double>(h, L.off_dfb);
  }
  if (o->precision == PNGF_RFORM) {
    for (int f = 0; f < F; ++f) {
      P.T0[f] = at<z64>(h, L.off_T[f]);
      P.Up[f] = at<z64>(h, L.off_Up[f]);
      P.alph[f] = at<z64>(h, L.off_ralph[f]);
    }
    P.pm = at<int32_t>(h, L.off_rpm);
    P.kcap = o->k_fold > 0 ? std::min(o->k_fold, pngf::kRPanel) : pngf::kRPanel;
    P.k_refresh = std::min(o->k_refresh, pngf::kWoodMax);
  }
  h->cinv_stale = false;
  // Zero the padded matrix storage once (padding columns are never read, but
  // keep them defined), then upload G.
  HIPCHK(h, hipMemsetAsync(h->ws, 0, L.total, h->stream));
  for (int f = 0; f < F; ++f) {
    int st;
    if (pec) {
      std::vector<cd> Gt(h->pc.freq[f].G);
      for (int m = 0; m < nd; ++m) Gt[size_t(m) * nd + m] -= 1.0;
      st = upload_matrix(h, P.G[f], Gt, nd);
      if (!st) HIPCHK(h, hipStreamSynchronize(h->stream));   // Gt is released next
    } else {
      st = upload_matrix(h, P.G[f], h->pc.freq[f].G, nd);
    }
    if (st) return st;
    HIPCHK(h, hipMemcpyAsync(at<z64>(h, L.off_b[f]), h->pc.freq[f].b.data(), nd * sizeof(z64),
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(at<z64>(h, L.off_god[f]), h->pc.freq[f].god.data(), nd * sizeof(z64),
                             hipMemcpyHostToDevice, h->stream));
  }
  if (o->precision == PNGF_MIXED)
    for (int f = 0; f < F; ++f) HIPCHK(h, pngf::launch_to_c64(P.G[f], P.G32[f], nd, h->ld, h->stream));
  // the persistent search's barrier words start at generation 0
  HIPCHK(h, hipMemsetAsync(at<int32_t>(h, L.off_pbar), 0, pngf::kPersistBarBytes, h->stream));
  {
    // the staging area holds a batch-end read (state .. design buffers), a
    // search's visiting orders and their ranks, or at a search's end its logs
    // and design; the index lists of an initial inverse follow in a region of
    // their own, which nothing else writes (staging stops at pin_idx)
    const size_t stage =
        pngf::kPinStage +
        std::max({L.off_bitsB + nd - L.off_state,
                  12 * size_t(std::max(1, o->max_accepts)) + size_t(nd) + 16,
                  pngf::kStageOrders + 2 * size_t(o->max_sweeps) * nd * sizeof(int32_t)});
    h->pin_idx = (stage + 255) & ~size_t(255);
    const size_t need = h->pin_idx + 3 * size_t(nd) * sizeof(int32_t);
    if (h->pin && h->pin_bytes < need) {
      (void)hipHostFree(h->pin);
      h->pin = nullptr;
    }
    if (!h->pin) {
      HIPCHK(h, hipHostMalloc(reinterpret_cast<void**>(&h->pin), need));
      h->pin_bytes = need;
    }
  }
  HIPCHK(h, hipMemsetAsync(at<int32_t>(h, L.off_flag), 0, sizeof(int32_t), h->stream));
  if (!h->ev_pin) HIPCHK(h, hipEventCreateWithFlags(&h->ev_pin, hipEventDisableTiming));
  if (!h->ev_ahead) HIPCHK(h, hipEventCreateWithFlags(&h->ev_ahead, hipEventDisableTiming));
  if (!h->ev_inv) HIPCHK(h, hipEventCreateWithFlags(&h->ev_inv, hipEventDisableTiming));
  HIPCHK(h, hipEventRecord(h->ev_pin, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->bound = true;
  h->have_design = false;
  return PNGF_OK;
}

int pngf_set_design(pngf_handle* h, const uint8_t* bits) {
  int st = check_ready(h, false);
  if (st) return st;
  if (!bits) return fail(h, PNGF_EINVAL, "null bits");
  const int nd = h->pc.n_d;
  for (int a = 0; a < nd; ++a) h->bits[a] = bits[a] ? 1 : 0;
  h->bits_fresh = false;
  HIPCHK(h, hipMemcpyAsync(h->P.bits, h->bits.data(), nd, hipMemcpyHostToDevice, h->stream));
  pngf::DbsState s{};
  s.m = -1;
  s.key = pngf::kNoKey;
  s.eta = h->opt.eta;
  st = write_state(h, &s);
  if (st) return st;
  h->have_design = false;
  // the unpivoted inverse is queued and checked when the handle is next used
  st = device_reinvert(h, true, true);
  if (st) return st;
  h->have_design = true;
  return PNGF_OK;
}

int pngf_evaluate(pngf_handle* h, double* f, double* x, double* e_d) {
  int st = check_ready(h, true);
  if (st) return st;
  pngf::DbsState s;
  st = read_state(h, &s);
  if (st) return st;
  const int F = int(h->pc.freq.size()), nd = h->pc.n_d;
  if (f) *f = s.f;
  if (x)
    for (int fi = 0; fi < F; ++fi) { x[2 * fi] = s.x[fi].re; x[2 * fi + 1] = s.x[fi].im; }
  if (e_d) {
    for (int fi = 0; fi < F; ++fi)
      HIPCHK(h, hipMemcpyAsync(e_d + size_t(fi) * 2 * nd, h->P.E[fi], nd * sizeof(z64),
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  return PNGF_OK;
}

int pngf_gradient(pngf_handle* h, double* grad) {
  int st = check_ready(h, true);
  if (st) return st;
  if (!grad) return fail(h, PNGF_EINVAL, "null output");
  if (h->pc.pec) return fail(h, PNGF_EINVAL, "no permittivity gradient for PEC pixels");
  double* d = at<double>(h, h->lay.off_df);
  HIPCHK(h, pngf::launch_gradient(h->P, d, h->stream));
  HIPCHK(h, hipMemcpyAsync(grad, d, h->pc.n_d * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

int pngf_flip_set(pngf_handle* h, const int32_t* pix, int32_t n) {
  int st = check_ready(h, true);
  if (st) return st;
  if (h->opt.precision == PNGF_MIXED)
    return fail(h, PNGF_EINVAL, "pixel sets need an FP64_PLAIN or RFORM handle");
  const int nd = h->pc.n_d;
  if (n < 0 || (n > 0 && !pix)) return fail(h, PNGF_EINVAL, "bad pixel list");
  std::vector<uint8_t> seen(nd, 0);
  for (int r = 0; r < n; ++r) {
    if (pix[r] < 0 || pix[r] >= nd) return fail(h, PNGF_EINVAL, "pixel out of range");
    if (seen[pix[r]]++) return fail(h, PNGF_EINVAL, "repeated pixel");
  }
  st = ensure_cinv(h);
  if (st) return st;
  if (n == 0) return PNGF_OK;
  HIPCHK(h, hipMemcpyAsync(h->bits.data(), h->P.bits, nd, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int r = 0; r < n; ++r) h->bits[pix[r]] ^= 1;
  HIPCHK(h, hipMemcpyAsync(h->P.bits, h->bits.data(), nd, hipMemcpyHostToDevice, h->stream));
  // blocks of at most kWoodMax pixels, each one exact rank-M update
  bool singular = false;
  for (int r0 = 0; r0 < n && !singular; r0 += pngf::kWoodMax) {
    std::vector<int32_t> blk(pix + r0, pix + std::min(n, r0 + pngf::kWoodMax));
    st = woodbury_update(h, blk, h->bits, &singular);
    if (st) return st;
  }
  st = singular ? device_reinvert(h) : reform_fields(h);
  if (st) return st;
  h->cinv_stale = false;
  return capture_ref_bits(h);
}

int pngf_score_flips(pngf_handle* h, const int32_t* cand, int32_t n, double* f_new) {
  int st = check_ready(h, true);
  if (st) return st;
  st = ensure_cinv(h);
  if (st) return st;
  if (n < 0 || n > h->pc.n_d || (n > 0 && (!cand || !f_new)))
    return fail(h, PNGF_EINVAL, "bad candidate list");
  for (int r = 0; r < n; ++r)
    if (cand[r] < 0 || cand[r] >= h->pc.n_d) return fail(h, PNGF_EINVAL, "candidate out of range");
  if (n == 0) return PNGF_OK;
  int32_t* dcand = at<int32_t>(h, h->lay.off_cand);
  HIPCHK(h, hipMemcpyAsync(dcand, cand, n * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, pngf::launch_score_rows(h->P, h->npl, dcand, n, nullptr, h->stream));
  std::vector<double> df(n);
  HIPCHK(h, hipMemcpyAsync(df.data(), h->P.df, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  pngf::DbsState s;
  st = read_state(h, &s);
  if (st) return st;
  for (int r = 0; r < n; ++r) f_new[r] = s.f + df[r];
  return PNGF_OK;
}

int pngf_accept_flips(pngf_handle* h, const int32_t* pix, int32_t n) {
  int st = check_ready(h, true);
  if (st) return st;
  st = ensure_cinv(h);
  if (st) return st;
  if (n < 0 || (n > 0 && !pix)) return fail(h, PNGF_EINVAL, "bad pixel list");
  for (int r = 0; r < n; ++r)
    if (pix[r] < 0 || pix[r] >= h->pc.n_d) return fail(h, PNGF_EINVAL, "pixel out of range");
  pngf::DbsState s;
  st = read_state(h, &s);
  if (st) return st;
  s.done = 0;
  s.n_sweeps = 0;
  st = write_state(h, &s);
  if (st) return st;
  // tau of the current state for every pixel (needed by the update scalars).
  HIPCHK(h, pngf::launch_score_rows(h->P, h->npl, nullptr, h->pc.n_d, nullptr, h->stream));
  for (int r = 0; r < n; ++r) {
    HIPCHK(h, pngf::launch_select_prep(h->P, pix[r], h->stream));
    HIPCHK(h, pngf::launch_accept_rescore(h->P, h->npl, h->stream));
    h->bits[pix[r]] ^= 1;
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

int pngf_refresh(pngf_handle* h) {
  int st = check_ready(h, true);
  if (st) return st;
  // The search bookkeeping in the device state is kept; x and f are re-formed.
  return device_reinvert(h);
}

int pngf_dbs_run(pngf_handle* h, const int32_t* perms, int32_t n_sweeps, int32_t* accepted,
                 double* f_trace, pngf_dbs_result* res) {
  int st = dbs_prologue(h, perms, n_sweeps);
  if (st) return st;
  // the uploads above are queued behind a deferred initial inverse; its
  // check comes now, and a re-inversion means starting the state again
  bool redone = false;
  st = settle_inverse(h, &redone);
  if (st) return st;
  if (redone) {
    st = dbs_prologue(h, perms, n_sweeps);
    if (st) return st;
  }
  // the state reads of the search land in the handle's pinned scratch
  auto* pinned = reinterpret_cast<pngf::DbsState*>(h->pin + pngf::kPinState);
  int64_t n_refresh = 0, n_band = 0;
  int rc = (h->opt.precision == PNGF_MIXED)   ? run_mixed(h, pinned, &n_refresh, &n_band)
           : (h->opt.precision == PNGF_RFORM) ? run_rform(h, pinned)
                                              : run_plain(h, pinned);
  pngf::DbsState fin = *pinned;
  if (rc) return rc;
  return dbs_epilogue(h, fin, n_refresh, n_band, accepted, f_trace, res);
}

int pngf_tile_dbs_run(pngf_handle* h, const int32_t* tiles, int32_t n_tiles, int32_t m,
                      const int32_t* perms, int32_t n_sweeps, int32_t* accepted, double* f_trace,
                      pngf_dbs_result* res) {
  int st = check_ready(h, true);
  if (st) return st;
  const int nd = h->pc.n_d;
  if (h->opt.precision != PNGF_FP64_PLAIN)
    return fail(h, PNGF_EINVAL, "the tile search runs on an FP64_PLAIN handle");
  if (m < 1 || m > h->opt.max_tile)
    return fail(h, PNGF_EINVAL, "tile size must be in [1, max_tile]");
  if (!tiles || n_tiles < 1 || n_tiles > nd) return fail(h, PNGF_EINVAL, "n_tiles must be in [1, n_d]");
  const size_t mr = size_t(pngf::tile_rows(m));
  const size_t cap = size_t(nd) * pngf::kTilePartPerPixel;
  if (size_t(n_tiles) * mr * mr > cap)
    return fail(h, PNGF_EINVAL, "n_tiles * Mpad^2 must not exceed 512 n_d (Mpad = 16, 32 or 64)");
  // K slices per tile block: enough workgroups to stream the whole chip
  const int nchunk = (nd + 31) / 32;
  const int ks = int(std::max<size_t>(1, std::min<size_t>({size_t(pngf::kTileSlicesMax),
      cap / (size_t(n_tiles) * mr * mr), size_t(nchunk), size_t((4096 + n_tiles - 1) / n_tiles)})));
  if (!perms || n_sweeps < 1 || n_sweeps > h->opt.max_sweeps)
    return fail(h, PNGF_EINVAL, "n_sweeps must be in [1, max_sweeps]");
  std::vector<std::vector<int32_t>> members(n_tiles);
  {
    std::vector<int32_t> seen(nd, -1);
    for (int t = 0; t < n_tiles; ++t) {
      bool pad = false;
      for (int c = 0; c < m; ++c) {
        const int32_t p = tiles[size_t(t) * m + c];
        if (p == -1) { pad = true; continue; }
        if (pad || p < 0 || p >= nd || seen[p] == t)
          return fail(h, PNGF_EINVAL, "tiles: distinct pixel ids, -1 only as trailing padding");
        seen[p] = t;
        members[t].push_back(p);
      }
      if (members[t].empty()) return fail(h, PNGF_EINVAL, "tiles: every tile needs a pixel");
    }
    std::vector<int32_t> chk(n_tiles);
    for (int s = 0; s < n_sweeps; ++s) {
      std::fill(chk.begin(), chk.end(), 0);
      for (int q = 0; q < n_tiles; ++q) {
        const int32_t t = perms[size_t(s) * n_tiles + q];
        if (t < 0 || t >= n_tiles || chk[t]++)
          return fail(h, PNGF_EINVAL, "perms must hold permutations of the tile ids");
      }
    }
  }
  int32_t* dtiles = at<int32_t>(h, h->lay.off_tiles);
  double* ddf = at<double>(h, h->lay.off_df);
  HIPCHK(h, hipMemcpyAsync(dtiles, tiles, size_t(n_tiles) * m * sizeof(int32_t),
                           hipMemcpyHostToDevice, h->stream));
  for (int k = 0; k < KID_N; ++k) { h->ktime_ms[k] = 0.0; h->klaunch[k] = 0; }
  pngf::DbsState s0;
  st = read_state(h, &s0);
  if (st) return st;
  HIPCHK(h, hipMemcpyAsync(h->bits.data(), h->P.bits, nd, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  const double f0 = s0.f;
  double f = f0;
  const double eta = h->opt.eta;
  std::vector<double> df(n_tiles);
  std::vector<int32_t> acc_log;
  std::vector<double> f_log;
  int64_t attempts = 0;
  int sweeps = 0, n_reinv = 0;
  bool converged = false, fresh = false;
  // the sequential search of the paper: scores stay valid until an accept
  for (int s = 0; s < n_sweeps && !converged; ++s) {
    if (int(acc_log.size()) >= h->opt.max_accepts) break;
    sweeps = s + 1;
    bool any = false;
    int pos = 0;
    while (pos < n_tiles) {
      if (!fresh) {
        Timer t(h, KID_TILE);
        HIPCHK(h, pngf::launch_tile_score(h->P, dtiles, n_tiles, m, ks,
                                          at<z64>(h, h->lay.off_tpart), ddf, h->stream));
        t.end();
        HIPCHK(h, hipMemcpyAsync(df.data(), ddf, n_tiles * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        fresh = true;
      }
      int q = pos;
      for (; q < n_tiles; ++q) {
        ++attempts;
        if (df[perms[size_t(s) * n_tiles + q]] > eta * f) break;
      }
      if (q == n_tiles) break;
      // accept tile perms[s][q]: flip its pixels, update C^-1, re-form fields
      const int32_t t = perms[size_t(s) * n_tiles + q];
      for (int32_t p : members[t]) h->bits[p] ^= 1;
      HIPCHK(h, hipMemcpyAsync(h->P.bits, h->bits.data(), nd, hipMemcpyHostToDevice, h->stream));
      bool singular = false;
      st = woodbury_update(h, members[t], h->bits, &singular);
      if (st) return st;
      if (singular) {
        st = device_reinvert(h);
        if (st) return st;
        ++n_reinv;
      } else {
        st = reform_fields(h);
        if (st) return st;
      }
      pngf::DbsState sn;
      st = read_state(h, &sn);
      if (st) return st;
      f = sn.f;
      if (!std::isfinite(f)) return fail(h, PNGF_ENUMERIC, "objective is not finite");
      acc_log.push_back(t);
      f_log.push_back(f);
      fresh = false;
      any = true;
      pos = q + 1;
      if (int(acc_log.size()) >= h->opt.max_accepts) break;
    }
    if (!any) converged = true;
  }
  if (h->opt.flags & (PNGF_FLAG_TIMING | PNGF_FLAG_TIMING_STEPS)) collect_times(h);
  const int na = int(acc_log.size());
  if (accepted && na) std::memcpy(accepted, acc_log.data(), na * sizeof(int32_t));
  if (f_trace && na) std::memcpy(f_trace, f_log.data(), na * sizeof(double));
  if (res) {
    res->n_accepted = na;
    res->sweeps = sweeps;
    res->converged = converged ? 1 : 0;
    res->n_refresh = n_reinv;
    res->attempts = attempts;
    res->n_verified = 0;
    res->f_initial = f0;
    res->f_final = f;
  }
  return PNGF_OK;
}

int pngf_force_singular_refresh(pngf_handle* h, int32_t n) {
  if (!h || n < 0) return PNGF_EINVAL;
  h->force_singular = n;
  return PNGF_OK;
}

int pngf_set_persist_spin(pngf_handle* h, int32_t polls) {
  if (!h || polls < 1) return PNGF_EINVAL;
  h->persist_spin = polls;
  return PNGF_OK;
}

int pngf_set_inverse_check(pngf_handle* h, double tol) {
  if (!h || !(tol >= 0.0)) return PNGF_EINVAL;
  h->np_tol = tol;
  return PNGF_OK;
}

int pngf_inverse_stats(pngf_handle* h, int64_t* unpivoted, int64_t* pivoted) {
  if (!h) return PNGF_EINVAL;
  if (h->inv_pending) {
    const int st = settle_inverse(h);
    if (st) return st;
  }
  if (unpivoted) *unpivoted = h->n_inv_np;
  if (pivoted) *pivoted = h->n_inv_piv;
  return PNGF_OK;
}

int pngf_kernel_times(pngf_handle* h, int32_t kid, double* total_ms, int64_t* launches) {
  if (!h || kid < 0 || kid >= KID_N) return PNGF_EINVAL;
  if (h->inv_pending) {
    const int st = settle_inverse(h);
    if (st) return st;
  }
  if (total_ms) *total_ms = h->ktime_ms[kid];
  if (launches) *launches = h->klaunch[kid];
  return PNGF_OK;
}

int pngf_destroy(pngf_handle* h) {
  if (!h) return PNGF_OK;
  if (h->inv_pending) (void)hipEventSynchronize(h->ev_inv);   // its copy lands in `pin`
  for (size_t k = 0; k + 2 < h->ev_pool.size(); k += 3) {
    hipEventDestroy(h->ev_pool[k]);
    hipEventDestroy(h->ev_pool[k + 1]);
  }
  for (hipEvent_t e : h->ev_free) hipEventDestroy(e);
  release_streams(h);
  if (h->pin) (void)hipHostFree(h->pin);
  if (h->ev_pin) (void)hipEventDestroy(h->ev_pin);
  if (h->ev_ahead) (void)hipEventDestroy(h->ev_ahead);
  if (h->ev_inv) (void)hipEventDestroy(h->ev_inv);
  delete h;
  return PNGF_OK;
}

}  // extern "C"


// ------------------------------------------------------------------ learned
namespace {

// Ranked search with chunks of one pixel, on the device: a direct binary
// search whose visiting order at every state is a fresh ranking (the network,
// or the first-order change), restarted from the top after each accept, so
// the first improving pixel of the ranking is accepted.  Runs on every form
// (FP64 plain, mixed with its FP64 decisions in the error band, R-form) with
// the same step kernels as pngf_dbs_run, all frequencies in each launch, and
// no host round trip per state.
int ranked_search(pngf_handle* h, pngf_model* m, int H, int W, int32_t max_accepts,
                  int32_t* accepted, double* f_trace, pngf_dbs_result* res) {
  const int nd = h->pc.n_d;
  if (max_accepts > h->opt.max_accepts)
    return fail(h, PNGF_EINVAL, "max_accepts exceeds the bound options' max_accepts");
  if (max_accepts == 0) {
    pngf::DbsState s;
    int st = read_state(h, &s);
    if (st) return st;
    if (res) {
      *res = pngf_dbs_result{};
      res->f_initial = res->f_final = s.f;
    }
    return PNGF_OK;
  }
  std::vector<int32_t> ident(nd);
  for (int i = 0; i < nd; ++i) ident[i] = i;
  int st = dbs_prologue(h, ident.data(), 1);
  if (st) return st;
  h->ranked = true;
  h->rank_model = m;
  h->rank_h = H;
  h->rank_w = W;
  const int32_t max_acc = h->P.max_acc;
  h->P.max_acc = max_accepts;
  auto* pinned = reinterpret_cast<pngf::DbsState*>(h->pin + pngf::kPinState);
  int64_t n_refresh = 0, n_band = 0;
  int rc = (h->opt.precision == PNGF_MIXED)   ? run_mixed(h, pinned, &n_refresh, &n_band)
           : (h->opt.precision == PNGF_RFORM) ? run_rform(h, pinned)
                                              : run_plain(h, pinned);
  pngf::DbsState fin = *pinned;
  h->ranked = false;
  h->rank_model = nullptr;
  h->P.max_acc = max_acc;
  if (rc) return rc;
  st = dbs_epilogue(h, fin, n_refresh, n_band, accepted, f_trace, res);
  if (st) return st;
  if (res) {
    // chunks scored beyond the first of each state (one per state visited)
    const int64_t states = int64_t(fin.n_acc) + (fin.converged ? 1 : 0);
    res->sweeps = int32_t(std::max<int64_t>(0, fin.attempts - states));
  }
  return PNGF_OK;
}


// Design region as an H x W rectangle in pixel order (needed by the CNN).
bool design_grid(pngf_handle* h, int* H, int* W) {
  const auto& dn = h->pc.design_nodes;
  const int nx = h->pc.grid.nx;
  int i0 = 1 << 30, i1 = -1, j0 = 1 << 30, j1 = -1;
  for (int64_t n : dn) {
    const int i = int(n % nx), j = int(n / nx);
    i0 = std::min(i0, i); i1 = std::max(i1, i);
    j0 = std::min(j0, j); j1 = std::max(j1, j);
  }
  *W = i1 - i0 + 1;
  *H = j1 - j0 + 1;
  return int64_t(*W) * *H == int64_t(dn.size());
}

}  // namespace

extern "C" {

int pngf_features(pngf_handle* h, float* X) {
  int st = check_ready(h, true);
  if (st) return st;
  if (!X) return fail(h, PNGF_EINVAL, "null output");
  int H = 0, W = 0;
  if (!design_grid(h, &H, &W)) return fail(h, PNGF_EINVAL, "design region is not a rectangle");
  float* d = at<float>(h, h->lay.off_feat);
  HIPCHK(h, pngf::launch_features(h->P, H, W, d, h->stream));
  HIPCHK(h, hipMemcpyAsync(X, d, size_t(kFeatChannels) * h->pc.n_d * sizeof(float),
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return PNGF_OK;
}

int pngf_learned_dbs_run(pngf_handle* h, pngf_model* m, int32_t k, int32_t max_accepts,
                         int32_t* accepted, double* f_trace, pngf_dbs_result* res) {
  int st = check_ready(h, true);
  if (st) return st;
  const int nd = h->pc.n_d;
  int H = 0, W = 0;
  if (!design_grid(h, &H, &W)) return fail(h, PNGF_EINVAL, "design region is not a rectangle");
  if (nd > 8192) return fail(h, PNGF_EINVAL, "the ranking holds at most 8192 pixels");
  if (m) {
    int mh = 0, mw = 0;
    if (pngf::model_hw(m, &mh, &mw) != PNGF_OK) return fail(h, PNGF_ESTATE, "model is not bound");
    if (mh != H || mw != W) return fail(h, PNGF_EINVAL, "model image size differs from the design");
    if (pngf::model_stream(m) != h->stream)
      return fail(h, PNGF_EINVAL, "model and handle must share the stream");
  }
  if (k < 1 || k > nd) return fail(h, PNGF_EINVAL, "k must be in [1, n_d]");
  if (max_accepts < 0) return fail(h, PNGF_EINVAL, "max_accepts must be >= 0");
  if (k == 1) return ranked_search(h, m, H, W, max_accepts, accepted, f_trace, res);
  if (h->opt.precision != PNGF_FP64_PLAIN)
    return fail(h, PNGF_EINVAL, "the learned search with k > 1 runs on an FP64 handle");
  pngf::DbsState s;
  st = read_state(h, &s);
  if (st) return st;
  const double f0 = s.f;
  s.done = 0;
  s.n_sweeps = 0;
  s.m = -1;
  s.eta = h->opt.eta;
  st = write_state(h, &s);
  if (st) return st;
  int32_t* d_rank = at<int32_t>(h, h->lay.off_cand);
  int32_t* d_best = at<int32_t>(h, h->lay.off_best);
  float* d_feat = at<float>(h, h->lay.off_feat);
  int64_t evals = 0, extra_chunks = 0;
  int n_acc = 0;
  bool converged = false;
  for (int k0 = 0; k0 < KID_N; ++k0) { h->ktime_ms[k0] = 0.0; h->klaunch[k0] = 0; }
  while (n_acc < max_accepts) {
    {
      // rank every pixel: by the network, or by the first-order change
      Timer t(h, KID_OTHER);
      const float* scores = nullptr;
      if (m) {
        float* y = nullptr;
        HIPCHK(h, pngf::model_score_state(m, h->P, &y));
        scores = y;
      } else {
        HIPCHK(h, pngf::launch_features(h->P, H, W, d_feat, h->stream));
        scores = d_feat + size_t(kFeatChannels - 1) * nd;
      }
      HIPCHK(h, pngf::launch_rank(scores, nd, d_rank, h->stream));
      t.end();
    }
    // exact scores of the ranking, k at a time, until a chunk improves
    int32_t best = -1;
    for (int c0 = 0; c0 < nd && best < 0; c0 += k) {
      const int n = std::min(k, nd - c0);
      {
        Timer t(h, KID_SCORE);
        HIPCHK(h, pngf::launch_score_rows(h->P, h->npl, d_rank + c0, n, nullptr, h->stream));
        HIPCHK(h, pngf::launch_pick_best(h->P.df, d_rank + c0, n, h->P.st, d_best, h->stream));
        t.end();
      }
      HIPCHK(h, hipMemcpyAsync(&best, d_best, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      evals += n;
      if (c0 > 0) extra_chunks += 1;
    }
    if (best < 0) { converged = true; break; }
    {
      Timer t(h, KID_ACCEPT);
      HIPCHK(h, pngf::launch_select_prep(h->P, best, h->stream));
      HIPCHK(h, pngf::launch_accept_only(h->P, h->npl, h->stream));
      t.end();
    }
    if (accepted) accepted[n_acc] = best;
    if (f_trace) {
      HIPCHK(h, hipMemcpyAsync(&f_trace[n_acc], &h->P.st->f, sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    }
    h->bits[best] ^= 1;
    n_acc += 1;
  }
  pngf::DbsState fin;
  st = read_state(h, &fin);
  if (st) return st;
  if (h->opt.flags & (PNGF_FLAG_TIMING | PNGF_FLAG_TIMING_STEPS)) collect_times(h);
  if (!std::isfinite(fin.f)) return fail(h, PNGF_ENUMERIC, "objective is not finite");
  if (res) {
    res->n_accepted = n_acc;
    res->sweeps = int32_t(extra_chunks);
    res->converged = converged ? 1 : 0;
    res->n_refresh = 0;
    res->attempts = evals;
    res->n_verified = 0;
    res->f_initial = f0;
    res->f_final = fin.f;
  }
  return PNGF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct pngf_batch {
  std::vector<pngf_handle*> hs;
  std::string err;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  pngf::ProbDev* d_probs = nullptr;
  int32_t* d_row0 = nullptr;            // [n+1] item offsets of the active problems
  int32_t* d_nact = nullptr;            // the active count the step kernel reads
  pngf::DbsState* d_states = nullptr;   // [2n]: A and B slot of every problem
  int npl = 1;
  int mixed = 0;
  int grid = 0;                         // 0 = one workgroup per work item
  int rpw = 2;                          // mixed: rows per wave (a work item is 4 rpw rows)
  bool bound = false;
  // captured 6-step graph for the launch shape (any active set)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_total = -1, g_grid = -1, g_rpw = -1;
  // autotuner record
  std::vector<int32_t> tune_grid, tune_rpw;
  std::vector<double> tune_work;        // streamed entries per step of each timed round
  std::vector<double> tune_ms;
  double last_ms_per_step = 0.0;
  // streams the refreshes of one round are spread over (default priority),
  // one join event each, and the event they start after
  std::vector<hipStream_t> rs;
  std::vector<hipEvent_t> rev;
  hipEvent_t ev_round = nullptr;
};

namespace {

int bfail(pngf_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg; else g_create_error = msg;
  return code;
}

#define BHIPCHK(b, call)                                                       \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return bfail(b, PNGF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t batch_bytes(int n) {
  return align256(size_t(n) * sizeof(pngf::ProbDev)) + align256(size_t(n + 2) * sizeof(int32_t)) +
         align256(size_t(2 * n) * sizeof(pngf::DbsState));
}

void drop_graph(pngf_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->g_total = b->g_grid = b->g_rpw = -1;
}

void release_refresh_streams(pngf_batch* b) {
  for (hipStream_t r : b->rs) (void)hipStreamDestroy(r);
  for (hipEvent_t e : b->rev) (void)hipEventDestroy(e);
  if (b->ev_round) (void)hipEventDestroy(b->ev_round);
  b->rs.clear();
  b->rev.clear();
  b->ev_round = nullptr;
}

// FP64 refreshes of several problems of a batch, in three parts.
// batch_refresh_fetch: their designs come up in one copy (one wait on the
// batch stream), and the refresh streams' start event is recorded there.
// pbits: pinned host memory for the designs (the sum of the problems' N_d
// bytes).
int batch_refresh_fetch(pngf_batch* b, const std::vector<int>& ref, uint8_t* pbits) {
  if (ref.empty()) return PNGF_OK;
  std::vector<size_t> boff;
  size_t off = 0;
  for (int p : ref) {
    pngf_handle* h = b->hs[p];
    boff.push_back(off);
    BHIPCHK(b, hipMemcpyAsync(pbits + off, h->P.bits, h->pc.n_d, hipMemcpyDeviceToHost, b->stream));
    off += size_t(h->pc.n_d);
  }
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  BHIPCHK(b, hipEventRecord(b->ev_round, b->stream));
  for (size_t j = 0; j < ref.size(); ++j) {
    pngf_handle* h = b->hs[ref[j]];
    h->bits.assign(pbits + boff[j], pbits + boff[j] + h->pc.n_d);
    h->bits_fresh = true;
  }
  return PNGF_OK;
}

// batch_refresh_launch: each problem's block-Woodbury update, field
// re-formation and (rescore) FP64 rescoring + band measurement are queued on
// one of the refresh streams, round-robin, after the fetch's event, so that
// the small kernels of different problems overlap each other and whatever
// the batch stream runs meanwhile (the host's issue time overlaps it too).
// Without rescore (the end of a search) only the FP64 state is re-formed.
// No wait: batch_refresh_settle.
int batch_refresh_launch(pngf_batch* b, const std::vector<int>& ref,
                         const std::vector<char>& meas, bool rescore) {
  if (ref.empty()) return PNGF_OK;
  const int K = std::min<int>(int(b->rs.size()), int(ref.size()));
  for (int k = 0; k < K; ++k) BHIPCHK(b, hipStreamWaitEvent(b->rs[k], b->ev_round, 0));
  for (size_t j = 0; j < ref.size(); ++j) {
    pngf_handle* h = b->hs[ref[j]];
    h->stream = b->rs[j % K];
    h->wood_pending = false;
    int st;
    if (rescore) {
      C64Pass c64pass(h);
      st = fp64_refresh(h, true, true);
    } else {
      st = fp64_refresh(h, true);
    }
    if (st == PNGF_OK && rescore) st = refresh_rescore(h, meas[j] != 0);
    if (st == PNGF_OK && !rescore && h->wood_pending) {
      int32_t* wst = reinterpret_cast<int32_t*>(h->pin + 24);
      *wst = 0;
      h->rescore_pending = true;
      if (hipMemcpyAsync(wst, at<int32_t>(h, h->lay.off_status), sizeof(int32_t),
                         hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        st = fail(h, PNGF_EDEVICE, "status read failed");
    }
    h->stream = b->stream;
    if (st) return bfail(b, st, "problem " + std::to_string(ref[j]) + ": " + h->err);
  }
  for (int k = 0; k < K; ++k) BHIPCHK(b, hipEventRecord(b->rev[k], b->rs[k]));
  return PNGF_OK;
}

// batch_refresh_settle: wait for the refreshes batch_refresh_launch queued,
// then let each problem
// take its band (or re-invert, on the batch stream, if its deferred update
// was singular).
int batch_refresh_settle(pngf_batch* b, const std::vector<int>& ref,
                         const std::vector<char>& meas, bool rescore) {
  if (ref.empty()) return PNGF_OK;
  const int K = std::min<int>(int(b->rs.size()), int(ref.size()));
  for (int k = 0; k < K; ++k) BHIPCHK(b, hipEventSynchronize(b->rev[k]));
  for (size_t j = 0; j < ref.size(); ++j) {
    pngf_handle* h = b->hs[ref[j]];
    int st = PNGF_OK;
    if (rescore) {
      st = refresh_settle(h, meas[j] != 0);
    } else {
      const bool singular = h->rescore_pending && *reinterpret_cast<const int32_t*>(h->pin + 24);
      h->rescore_pending = false;
      h->wood_pending = false;
      if (singular) st = device_reinvert(h);
    }
    if (st) return bfail(b, st, "problem " + std::to_string(ref[j]) + ": " + h->err);
  }
  return PNGF_OK;
}

// Upload the descriptors and item offsets of the active problems (and their
// count, which the step kernel reads on the device) and, for a new launch
// shape, capture the 6-step graph (one full cycle of state parity and key
// slot).  The graph does not depend on the active set.
int batch_items(const pngf_batch* b, int nd, int rpw) {
  // work items of one problem: rows (FP64), groups of 4 rpw rows (mixed)
  return b->mixed ? (nd + 4 * rpw - 1) / (4 * rpw) : nd;
}

int batch_prepare(pngf_batch* b, const std::vector<int>& active, int grid, int rpw) {
  const int n = int(active.size());
  if (n == 0) return PNGF_OK;
  std::vector<pngf::ProbDev> probs;
  std::vector<int32_t> row0(b->hs.size() + 2, 0);
  for (int q = 0; q < n; ++q) {
    const pngf_handle* h = b->hs[active[q]];
    probs.push_back(h->P);
    row0[q + 1] = row0[q] + batch_items(b, h->pc.n_d, rpw);
  }
  int total = 0;   // items of every problem (the launch covers any active set)
  for (const pngf_handle* h : b->hs) total += batch_items(b, h->pc.n_d, rpw);
  row0[b->hs.size() + 1] = n;   // d_nact follows d_row0[0..n_all]
  BHIPCHK(b, hipMemcpyAsync(b->d_probs, probs.data(), n * sizeof(pngf::ProbDev),
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->d_row0, row0.data(), row0.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  if (b->exec && b->g_total == total && b->g_grid == grid && b->g_rpw == rpw) return PNGF_OK;
  drop_graph(b);
  BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  for (int t = 0; t < 6; ++t) {
    hipError_t e = pngf::launch_batch_step(b->d_probs, b->d_row0, b->d_nact, total, grid, b->npl,
                                           b->mixed, rpw, t, b->stream);
    if (e != hipSuccess) {
      hipGraph_t g = nullptr;
      hipStreamEndCapture(b->stream, &g);
      if (g) hipGraphDestroy(g);
      return bfail(b, PNGF_EDEVICE, std::string("batch step capture: ") + hipGetErrorString(e));
    }
  }
  BHIPCHK(b, hipStreamEndCapture(b->stream, &b->graph));
  BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->g_total = total;
  b->g_grid = grid;
  b->g_rpw = rpw;
  return PNGF_OK;
}

}  // namespace

extern "C" {

int pngf_batch_create(pngf_handle* const* handles, int32_t n, pngf_batch** out) {
  if (!out) return bfail(nullptr, PNGF_EINVAL, "null output pointer");
  *out = nullptr;
  if (!handles || n < 1) return bfail(nullptr, PNGF_EINVAL, "need at least one handle");
  pngf_batch* b = new (std::nothrow) pngf_batch();
  if (!b) return bfail(nullptr, PNGF_ENOMEM, "out of host memory");
  for (int p = 0; p < n; ++p) {
    if (!handles[p]) { delete b; return bfail(nullptr, PNGF_EINVAL, "null handle in batch"); }
    for (int q = 0; q < p; ++q)
      if (handles[q] == handles[p]) { delete b; return bfail(nullptr, PNGF_EINVAL, "handle listed twice"); }
    b->hs.push_back(handles[p]);
  }
  *out = b;
  return PNGF_OK;
}

const char* pngf_batch_last_error(const pngf_batch* b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

int pngf_batch_workspace_bytes(pngf_batch* b, size_t* bytes) {
  if (!b || !bytes) return PNGF_EINVAL;
  *bytes = batch_bytes(int(b->hs.size()));
  return PNGF_OK;
}

int pngf_batch_bind(pngf_batch* b, void* dev_ws, size_t bytes, void* stream) {
  if (!b || !dev_ws) return PNGF_EINVAL;
  const int n = int(b->hs.size());
  if (bytes < batch_bytes(n)) return bfail(b, PNGF_ENOMEM, "batch workspace too small");
  if (reinterpret_cast<uintptr_t>(dev_ws) & 255)
    return bfail(b, PNGF_EINVAL, "workspace must be 256-byte aligned");
  if (stream == nullptr)
    return bfail(b, PNGF_EINVAL, "a batch needs a non-default stream (graph capture)");
  int npl = 1;
  const int prec = b->hs[0]->opt.precision;
  for (pngf_handle* h : b->hs) {
    if (!h->bound) return bfail(b, PNGF_ESTATE, "every handle must be bound");
    if (h->opt.precision != prec) return bfail(b, PNGF_EINVAL, "mixed precisions in one batch");
    if (h->opt.precision == PNGF_RFORM)
      return bfail(b, PNGF_EINVAL, "batches run FP64 plain or mixed handles");
    if (h->stream != static_cast<hipStream_t>(stream))
      return bfail(b, PNGF_EINVAL, "every handle must be bound to the batch stream");
    npl = std::max(npl, h->npl);
  }
  drop_graph(b);
  if (b->rs.empty()) {
    for (int k = 0; k < pngf::kBatchRefreshStreams; ++k) {
      hipStream_t r = nullptr;
      hipEvent_t e = nullptr;
      BHIPCHK(b, hipStreamCreateWithFlags(&r, hipStreamNonBlocking));
      b->rs.push_back(r);
      BHIPCHK(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->rev.push_back(e);
    }
    BHIPCHK(b, hipEventCreateWithFlags(&b->ev_round, hipEventDisableTiming));
  }
  b->ws = static_cast<char*>(dev_ws);
  b->ws_bytes = bytes;
  b->stream = static_cast<hipStream_t>(stream);
  size_t off = 0;
  b->d_probs = reinterpret_cast<pngf::ProbDev*>(b->ws + off);
  off += align256(size_t(n) * sizeof(pngf::ProbDev));
  b->d_row0 = reinterpret_cast<int32_t*>(b->ws + off);
  b->d_nact = b->d_row0 + n + 1;
  off += align256(size_t(n + 2) * sizeof(int32_t));
  b->d_states = reinterpret_cast<pngf::DbsState*>(b->ws + off);
  b->npl = npl;
  b->mixed = (prec == PNGF_MIXED) ? 1 : 0;
  b->bound = true;
  return PNGF_OK;
}

int pngf_batch_set_grid(pngf_batch* b, int32_t grid) {
  if (!b || grid < 0) return PNGF_EINVAL;
  b->grid = grid;
  return PNGF_OK;
}

int pngf_batch_tuning(pngf_batch* b, int32_t* grids, int32_t* rows, double* ms_per_step,
                      int32_t cap, int32_t* n) {
  if (!b || !n) return PNGF_EINVAL;
  *n = int32_t(b->tune_grid.size());
  for (int k = 0; k < std::min<int>(cap, *n); ++k) {
    if (grids) grids[k] = b->tune_grid[k];
    if (rows) rows[k] = b->mixed ? 4 * b->tune_rpw[k] : 1;
    if (ms_per_step) ms_per_step[k] = b->tune_ms[k];
  }
  return PNGF_OK;
}

int pngf_batch_dbs_run(pngf_batch* b, const int32_t* const* perms, const int32_t* n_sweeps,
                       int32_t* const* accepted, double* const* f_trace,
                       pngf_dbs_result* results, int32_t autotune) {
  if (!b || !b->bound) return bfail(b, PNGF_ESTATE, "batch is not bound");
  if (!perms || !n_sweeps) return bfail(b, PNGF_EINVAL, "null perms / n_sweeps");
  const int n = int(b->hs.size());
  std::vector<int64_t> nref(n, 0), nband(n, 0);
  // every problem's initial inverse checked first
  for (int p = 0; p < n; ++p) {
    pngf_handle* h = b->hs[p];
    int st = check_ready(h, true);
    if (st) return bfail(b, st, std::string("problem ") + std::to_string(p) + ": " + h->err);
  }
  // per-problem start: prologue, FP32 copies (mixed), scoring into key slot 0
  for (int p = 0; p < n; ++p) {
    pngf_handle* h = b->hs[p];
    int st = dbs_prologue(h, perms[p], n_sweeps[p]);
    if (st) return bfail(b, st, std::string("problem ") + std::to_string(p) + ": " + h->err);
    if (b->mixed) {
      st = capture_ref_bits(h);
      if (st) return bfail(b, st, h->err);
      for (int f = 0; f < int(h->pc.freq.size()); ++f)
        BHIPCHK(b, pngf::launch_to_c64(h->P.Cinv[f], h->P.C0[f], h->pc.n_d, h->ld, b->stream));
      pngf::DbsState s;
      st = read_state(h, &s);
      if (st) return bfail(b, st, h->err);
      s.kpanel = 0;
      s.n_since = 0;
      s.exact = 1;
      s.n_band = 0;
      st = write_state(h, &s);
      if (st) return bfail(b, st, h->err);
    }
    st = start_segment(h);
    if (st) return bfail(b, st, h->err);
  }
  // move every state into the batch slots (A = 2p, B = 2p+1)
  std::vector<pngf::DbsState*> own_a(n), own_b(n);
  for (int p = 0; p < n; ++p) {
    pngf_handle* h = b->hs[p];
    own_a[p] = h->P.st;
    own_b[p] = h->P.stB;
    BHIPCHK(b, hipMemcpyAsync(&b->d_states[2 * p], h->P.st, sizeof(pngf::DbsState),
                              hipMemcpyDeviceToDevice, b->stream));
    h->P.st = &b->d_states[2 * p];
    h->P.stB = &b->d_states[2 * p + 1];
  }
  // descriptors in decreasing order of a step's work (N_d^2 x frequencies),
  // so that the largest problems' work items are dispatched first and the
  // small ones fill in behind them
  auto by_work = [&](int p, int q) {
    const double wp = double(b->hs[p]->pc.n_d) * b->hs[p]->pc.n_d * b->hs[p]->pc.freq.size();
    const double wq = double(b->hs[q]->pc.n_d) * b->hs[q]->pc.n_d * b->hs[q]->pc.freq.size();
    return wp != wq ? wp > wq : p < q;
  };
  std::vector<int> active(n);
  for (int p = 0; p < n; ++p) active[p] = p;
  std::sort(active.begin(), active.end(), by_work);
  pngf::DbsState* host_states = nullptr;
  BHIPCHK(b, hipHostMalloc(reinterpret_cast<void**>(&host_states), 2 * n * sizeof(pngf::DbsState)));
  size_t sum_nd = 0;
  for (pngf_handle* h : b->hs) sum_nd += size_t(h->pc.n_d);
  uint8_t* pbits = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&pbits), sum_nd) != hipSuccess) {
    hipHostFree(host_states);
    return bfail(b, PNGF_ENOMEM, "pinned host memory for the designs");
  }
  int rc = PNGF_OK;
  // autotuner: candidate launch shapes, each timed on one 6-step replay of
  // the live search (every shape gives bitwise the same per-row arithmetic)
  // (grid, rows per wave); the mixed step also tries one row per wave (work
  // items of four rows: twice the workgroups, each reading g_m per row)
  std::vector<std::pair<int, int>> cand;
  if (autotune) {
    for (int rp : b->mixed ? std::vector<int>{2, 1} : std::vector<int>{2})
      for (int g : {0, 8192, 4096, 2048, 1024}) cand.emplace_back(g, rp);
    b->tune_grid.clear();
    b->tune_rpw.clear();
    b->tune_ms.clear();
    b->tune_work.clear();
  }
  size_t ci = 0;
  int grid = b->grid, rpw = b->rpw;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  int64_t max_rounds = 0;
  for (pngf_handle* h : b->hs) max_rounds = std::max<int64_t>(max_rounds, 4 * int64_t(h->opt.max_accepts) + 64);
  // A problem that needs a refresh sits out one round: its refresh is queued
  // on the refresh streams just after that round's steps (it runs beside
  // them, and so does the host's issue time), settled after them, and the
  // problem rejoins the round after (its own sequence does not depend on
  // when its steps run).
  std::vector<int> toissue, inflight;
  std::vector<char> toissue_meas, inflight_meas;
  for (int64_t round = 0; round < max_rounds && !(active.empty() && toissue.empty()); ++round) {
    const bool stepping = !active.empty();
    const bool tuning = stepping && ci < cand.size();
    int reps = 0;
    if (stepping) {
      if (tuning) {
        grid = cand[ci].first;
        rpw = cand[ci].second;
      }
      rc = batch_prepare(b, active, grid, rpw);
      if (rc) break;
      hipEventRecord(e0, b->stream);
      reps = tuning ? 1 : 5;   // 30 steps per round: about one refresh interval
      for (int r = 0; r < reps && rc == PNGF_OK; ++r) {
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) rc = bfail(b, PNGF_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
      }
      if (rc) break;
      hipEventRecord(e1, b->stream);
      if (hipMemcpyAsync(host_states, b->d_states, 2 * n * sizeof(pngf::DbsState),
                         hipMemcpyDeviceToHost, b->stream) != hipSuccess) {
        rc = bfail(b, PNGF_EDEVICE, "state read failed");
        break;
      }
    }
    // the refreshes decided last round, beside this round's steps
    rc = batch_refresh_launch(b, toissue, toissue_meas, true);
    if (rc) break;
    inflight.swap(toissue);
    inflight_meas.swap(toissue_meas);
    toissue.clear();
    toissue_meas.clear();
    if (stepping) {
      const hipError_t e = hipStreamSynchronize(b->stream);
      if (e != hipSuccess) { rc = bfail(b, PNGF_EDEVICE, hipGetErrorString(e)); break; }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      b->last_ms_per_step = ms / (6.0 * reps);
      if (tuning) {
        // the active set differs from round to round (problems sit out for
        // their refreshes), so shapes are compared per streamed entry: a
        // step reads N_d^2 entries of every active frequency
        double work = 0.0;
        for (int q : active) {
          const pngf_handle* h = b->hs[q];
          work += double(h->pc.n_d) * h->pc.n_d * double(h->pc.freq.size());
        }
        b->tune_grid.push_back(cand[ci].first);
        b->tune_rpw.push_back(cand[ci].second);
        b->tune_ms.push_back(ms / 6.0);
        b->tune_work.push_back(work);
        if (++ci == cand.size()) {
          size_t best = 0;
          for (size_t k = 1; k < b->tune_ms.size(); ++k)
            if (b->tune_ms[k] / b->tune_work[k] < b->tune_ms[best] / b->tune_work[best]) best = k;
          b->grid = grid = b->tune_grid[best];
          b->rpw = rpw = b->tune_rpw[best];
        }
      }
    }
    rc = batch_refresh_settle(b, inflight, inflight_meas, true);
    if (rc) break;
    std::vector<int> back;
    back.swap(inflight);
    inflight_meas.clear();
    std::vector<int> next;
    for (int p : active) {
      pngf_handle* h = b->hs[p];
      pngf::DbsState& s = host_states[2 * p];
      if (normalize(h, &s)) { rc = bfail(b, PNGF_EDEVICE, h->err); break; }
      if (s.done) continue;
      if (b->mixed) {
        bool refresh = s.need_refresh != 0;
        const bool band_hit = s.need_refresh == 2;
        if (!refresh && h->opt.k_refresh == 0 && !s.exact && s.n_since >= pngf::kDriftEvery) {
          double ratio = 0.0;
          if (mixed_residual(h, &ratio)) { rc = bfail(b, PNGF_EDEVICE, h->err); break; }
          refresh = ratio > pngf::kDriftTol;
        }
        if (refresh) {
          toissue.push_back(p);
          toissue_meas.push_back(s.exact ? 0 : 1);
          nref[p] += 1;
          if (band_hit) nband[p] += 1;
          continue;
        }
        if (s.kpanel >= pngf::kPanelCap - 12 ||
            (h->opt.k_fold > 0 && s.kpanel >= h->opt.k_fold)) {
          for (int f = 0; f < int(h->pc.freq.size()); ++f) {
            if (pngf::launch_fold_q(h->P, f, s.kpanel, b->stream) != hipSuccess ||
                pngf::launch_fold(h->P, f, s.kpanel, b->stream) != hipSuccess) {
              rc = bfail(b, PNGF_EDEVICE, "fold launch failed");
              break;
            }
          }
          if (rc) break;
          s.kpanel = 0;
          if (write_state(h, &s)) { rc = bfail(b, PNGF_EDEVICE, h->err); break; }
        }
      }
      next.push_back(p);
    }
    if (rc) break;
    rc = batch_refresh_fetch(b, toissue, pbits);
    if (rc) break;
    // descriptors keep their order (they are re-uploaded every round)
    next.insert(next.end(), back.begin(), back.end());
    std::sort(next.begin(), next.end(), by_work);
    active.swap(next);
  }
  if (rc) {
    // leave no refresh running on the handles' memory
    for (hipStream_t r : b->rs) (void)hipStreamSynchronize(r);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == PNGF_OK && !(active.empty() && toissue.empty()))
    rc = bfail(b, PNGF_ENUMERIC, "batch search did not terminate");
  // final FP64 state (mixed), results, and states back to each handle
  if (rc == PNGF_OK && b->mixed) {
    std::vector<int> all(n);
    for (int p = 0; p < n; ++p) all[p] = p;
    const std::vector<char> none(n, 0);
    rc = batch_refresh_fetch(b, all, pbits);
    if (rc == PNGF_OK) rc = batch_refresh_launch(b, all, none, false);
    if (rc == PNGF_OK) rc = batch_refresh_settle(b, all, none, false);
    if (rc) for (hipStream_t r : b->rs) (void)hipStreamSynchronize(r);
  }
  for (int p = 0; p < n && rc == PNGF_OK; ++p) {
    pngf_handle* h = b->hs[p];
    pngf::DbsState fin;
    if (read_state(h, &fin)) { rc = bfail(b, PNGF_EDEVICE, h->err); break; }
    if (dbs_epilogue(h, fin, nref[p], nband[p], accepted ? accepted[p] : nullptr,
                     f_trace ? f_trace[p] : nullptr, results ? &results[p] : nullptr)) {
      rc = bfail(b, PNGF_ENUMERIC, h->err);
      break;
    }
  }
  for (int p = 0; p < n; ++p) {
    pngf_handle* h = b->hs[p];
    if (h->P.st != own_a[p])
      hipMemcpyAsync(own_a[p], h->P.st, sizeof(pngf::DbsState), hipMemcpyDeviceToDevice, b->stream);
    h->P.st = own_a[p];
    h->P.stB = own_b[p];
  }
  hipStreamSynchronize(b->stream);
  hipHostFree(host_states);
  hipHostFree(pbits);
  return rc;
}

int pngf_batch_ms_per_step(pngf_batch* b, double* ms) {
  if (!b || !ms) return PNGF_EINVAL;
  *ms = b->last_ms_per_step;
  return PNGF_OK;
}

int pngf_batch_destroy(pngf_batch* b) {
  if (!b) return PNGF_OK;
  drop_graph(b);
  release_refresh_streams(b);
  delete b;
  return PNGF_OK;
}

}  // extern "C"
