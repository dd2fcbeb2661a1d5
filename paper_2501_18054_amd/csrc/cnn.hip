// Flip-proposal CNN of libpngf (gfx950): features from the PNGF state, a
// 4-layer 3x3 convolutional network (7 -> 32 -> 32 -> 32 -> 1, ReLU) trained
// and evaluated by hand-written kernels, BF16 operands on the matrix cores
// with FP32 accumulation, FP32 master weights and Adam.
//
// The network only ranks pixels; every accepted flip is decided by an exact
// PNGF evaluation (the paper's point against surrogate models: evaluations
// are exact, Results, Numerical Green's functions).
//
// Convolution as an implicit GEMM on v_mfma_f32_16x16x16bf16_1k: a wave owns
// 16 output pixels (along x) x 16 output channels; the K dimension is
// (input channel, ky, kx) padded to a multiple of 16, gathered on the fly from
// the activations (zero padding at the image border).  Operand layouts
// (16x16x16): lane l holds A[l%16][4(l/16)+v] and B[4(l/16)+v][l%16], v < 4;
// accumulator register r holds D[4(l/16)+r][l%16].  The data gradient is the
// same convolution with the flipped, transposed weights; the weight gradient
// is a GEMM over pixels (M = output channel, N = K, K = pixels): each chunk of
// pixels writes its partial tile, and a second pass adds the chunks in a fixed
// order, so training is bit-for-bit reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "dev_state.h"
#include "../../include/pngf.h"

namespace pngf {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 4;
constexpr int kCh[kLayers + 1] = {7, 32, 32, 32, 1};

__host__ __device__ inline int pad16(int x) { return (x + 15) & ~15; }

__device__ __forceinline__ short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return short(u >> 16);
}

// Y[n,o,y,x] = b[o] + sum_k Wb[o][k] * in(n, k, y, x), k = (c, ky, kx).
// in = relu(X) if relu_in.  gate != nullptr: Y *= (gate > 0) (ReLU backward).
__global__ __launch_bounds__(256) void k_conv(const float* X, int Cin, int relu_in,
                                              const short* Wb, int Kpad, const float* bias,
                                              float* Y, int Cout, int N, int H, int W,
                                              const float* gate) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int xt = (W + 15) / 16, ot = pad16(Cout) / 16;
  const int total = N * H * xt * ot;
  if (wave >= total) return;
  int t = wave;
  const int ob = t % ot; t /= ot;
  const int xb = t % xt; t /= xt;
  const int y = t % H;
  const int n = t / H;
  const int x0 = xb * 16, o0 = ob * 16;
  const int px = x0 + (lane & 15);        // A row: output pixel
  const int oc = o0 + (lane & 15);        // B column: output channel
  const int kq = 4 * (lane >> 4);
  const int K = Cin * 9;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Kpad; k0 += 16) {
    s4 a, b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + kq + v;
      float val = 0.f;
      if (k < K && px < W) {
        const int c = k / 9, r = k % 9;
        const int yy = y + r / 3 - 1, xx = px + r % 3 - 1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
          val = X[((size_t(n) * Cin + c) * H + yy) * W + xx];
          if (relu_in) val = fmaxf(val, 0.f);
        }
      }
      a[v] = to_bf16(val);
      b[v] = Wb[size_t(oc) * Kpad + k];   // padded rows/columns hold 0
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int o = o0 + (lane & 15);
  if (o >= Cout) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int x = x0 + 4 * (lane >> 4) + r;
    if (x >= W) continue;
    const size_t idx = ((size_t(n) * Cout + o) * H + y) * W + x;
    float v = acc[r] + (bias ? bias[o] : 0.f);
    if (gate && !(gate[idx] > 0.f)) v = 0.f;
    Y[idx] = v;
  }
}

// Partial weight / bias gradients of one chunk of pixels pc:
//   part[pc][o*K + k] = sum over the chunk of dZ[n,o,p] * in(n, k, p),
//   part[pc][Cout*K + o] = sum over the chunk of dZ[n,o,p]   (k-tile 0),
// k = (c, ky, kx), in = relu(X) if relu_in.  Every entry is written once.
__global__ __launch_bounds__(256) void k_wgrad(const float* dZ, const float* X, int Cin,
                                               int relu_in, int Cout, int N, int H, int W,
                                               float* part, int Kpad, int chunk) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ot = pad16(Cout) / 16, kt = Kpad / 16;
  const int P = N * H * W;
  const int nchunk = (P + chunk - 1) / chunk;
  const int total = ot * kt * nchunk;
  if (wave >= total) return;
  int t = wave;
  const int kb = t % kt; t /= kt;
  const int ob = t % ot;
  const int pc = t / ot;
  const int o = ob * 16 + (lane & 15);        // A row
  const int kcol = kb * 16 + (lane & 15);     // B column
  const int K = Cin * 9;
  const int c = kcol / 9, r = kcol % 9;
  const int dy = r / 3 - 1, dx = r % 3 - 1;
  const int q = 4 * (lane >> 4);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int p_end = min(P, (pc + 1) * chunk);
  for (int p0 = pc * chunk; p0 < p_end; p0 += 16) {
    s4 a, b;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = p0 + q + v;
      float av = 0.f, bv = 0.f;
      if (p < p_end) {
        const int x = p % W, yy0 = (p / W) % H, n = p / (W * H);
        if (o < Cout) av = dZ[((size_t(n) * Cout + o) * H + yy0) * W + x];
        if (kcol < K) {
          const int yy = yy0 + dy, xx = x + dx;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
            bv = X[((size_t(n) * Cin + c) * H + yy) * W + xx];
            if (relu_in) bv = fmaxf(bv, 0.f);
          }
        }
      }
      a[v] = to_bf16(av);
      b[v] = to_bf16(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // D[i][j] = dW[o0 + i][k0 + j], i = 4(l/16)+r, j = l%16
  float* pp = part + size_t(pc) * (size_t(Cout) * K + Cout);
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int oi = ob * 16 + 4 * (lane >> 4) + rr;
    const int kj = kb * 16 + (lane & 15);
    if (oi < Cout && kj < K) pp[size_t(oi) * K + kj] = acc[rr];
  }
  // bias gradient (FP32), once per (output tile, chunk): lanes of the first
  // k-tile sum their output channel over the chunk
  if (kb == 0 && lane < 16 && o < Cout) {
    for (int p = pc * chunk; p < p_end; ++p) {
      const int x = p % W, yy0 = (p / W) % H, n = p / (W * H);
      bsum += dZ[((size_t(n) * Cout + o) * H + yy0) * W + x];
    }
    pp[size_t(Cout) * K + o] = bsum;
  }
}

// g[e] = sum over chunks pc = 0, 1, ... of part[pc][e], in that order
// (e < n = Cout*K + Cout: the layer's weights, then its biases).
__global__ __launch_bounds__(256) void k_wsum(const float* part, int n, int nchunk, float* g) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int pc = 0; pc < nchunk; ++pc) s += part[size_t(pc) * n + e];
  g[e] = s;
}

// dY = clip(Y - T, -1, 1) / count (Huber, delta 1) and the loss sum of
// each workgroup in loss[blockIdx.x] (added in order by the host).
__global__ __launch_bounds__(256) void k_huber(const float* Y, const float* T, float* dY, int n,
                                               float inv_count, double* loss) {
  __shared__ double red[4];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (i < n) {
    const float r = Y[i] - T[i];
    const float a = fabsf(r);
    l = a <= 1.f ? 0.5 * double(r) * r : double(a) - 0.5;
    dY[i] = fminf(fmaxf(r, -1.f), 1.f) * inv_count;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) loss[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Adam on the flat FP32 parameters (Kingma & Ba).
__global__ __launch_bounds__(256) void k_adam(float* w, const float* g, float* m, float* v, int n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of layer l: Wb[o][c*9+r] and the flipped transpose
// Wt[c][o*9 + (8-r)] (data-gradient weights).
__global__ __launch_bounds__(256) void k_pack(const float* Wl, int Cin, int Cout, short* Wb,
                                              int Kpad, short* Wt, int Ktpad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= Cout * Cin * 9) return;
  const int o = e / (Cin * 9), k = e % (Cin * 9);
  const int c = k / 9, r = k % 9;
  const short b = to_bf16(Wl[e]);
  Wb[size_t(o) * Kpad + k] = b;
  if (Wt) Wt[size_t(c) * Ktpad + o * 9 + (8 - r)] = b;
}

// Zero n 32-bit words (a fill kernel rather than a memset node, so the
// allocation-free forward can be captured in a graph).
__global__ __launch_bounds__(256) void k_zero_words(uint32_t* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// CNN inputs of the current PNGF state for an H x W pixel grid (pixel m at
// y = m / W, x = m % W), seven channels:
//   bit, Re E / max|E|, Im E / max|E|, Re R' / max|R'|, Im R' / max|R'|,
//   |G_mm| / max|G_mm|, asinh(df_lin / (s f)),
// E, R', G_mm at the first frequency; df_lin is the flip's objective change
// with the denominator of eq. lru_eobj_rs set to 1 (first-order field change
// k0^2 delta E[m] R'[m]), summed over frequencies; s = kFeatScale.  The last
// channel alone is also the non-learned ranking.  One workgroup.
constexpr double kFeatScale = 1e-3;

__global__ __launch_bounds__(1024) void k_features(ProbDev P, int H, int W, float* X) {
  __shared__ double red[48];
  __shared__ double s_e, s_r, s_g;
  const int n = P.nd;
  double me = 0.0, mr = 0.0, mg = 0.0;
  for (int m = threadIdx.x; m < n; m += 1024) {
    me = fmax(me, zabs2(P.E[0][m]));
    mr = fmax(mr, zabs2(P.Rp[0][m]));
    mg = fmax(mg, zabs2(P.G[0][size_t(m) * P.ld + m]));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    me = fmax(me, __shfl_xor(me, o, 64));
    mr = fmax(mr, __shfl_xor(mr, o, 64));
    mg = fmax(mg, __shfl_xor(mg, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = me;
    red[16 + (threadIdx.x >> 6)] = mr;
    red[32 + (threadIdx.x >> 6)] = mg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int w = 0; w < 16; ++w) {
      a = fmax(a, red[w]);
      b = fmax(b, red[16 + w]);
      c = fmax(c, red[32 + w]);
    }
    s_e = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
    s_r = b > 0.0 ? 1.0 / sqrt(b) : 0.0;
    s_g = c > 0.0 ? 1.0 / sqrt(c) : 0.0;
  }
  __syncthreads();
  const DbsState* st = P.st;
  const double inv_f = st->f > 0.0 ? 1.0 / (kFeatScale * st->f) : 0.0;
  const size_t HW = size_t(H) * W;
  for (int m = threadIdx.x; m < n; m += 1024) {
    const z64 e = P.E[0][m], r = P.Rp[0][m];
    const double delta = P.bits[m] ? -P.deps : P.deps;
    double dfl = 0.0;
    for (int f = 0; f < P.nfreq; ++f) {
      const z64 dx = zscale(zmul(P.E[f][m], P.Rp[f][m]), P.k0sq[f] * delta);
      const z64 x = st->x[f];
      dfl += P.coef[f] * (2.0 * (x.re * dx.re + x.im * dx.im) + zabs2(dx));
    }
    X[m] = P.bits[m] ? 1.f : 0.f;
    X[HW + m] = float(e.re * s_e);
    X[2 * HW + m] = float(e.im * s_e);
    X[3 * HW + m] = float(r.re * s_r);
    X[4 * HW + m] = float(r.im * s_r);
    X[5 * HW + m] = float(sqrt(zabs2(P.G[0][size_t(m) * P.ld + m])) * s_g);
    X[6 * HW + m] = float(asinh(dfl * inv_f));
  }
}

// Ranking of n <= 8192 scores, best first (ties by index): bitonic sort of
// (score, index) pairs in LDS; out[0..n) receives the indices.  One
// workgroup.
__global__ __launch_bounds__(1024) void k_rank(const float* s, int n, int32_t* out) {
  __shared__ float v[8192];
  __shared__ int id[8192];
  int L = 1;
  while (L < n) L <<= 1;
  for (int i = threadIdx.x; i < L; i += 1024) {
    v[i] = i < n ? s[i] : -INFINITY;
    id[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= L; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < L; i += 1024) {
        const int j = i ^ stride;
        if (j > i) {
          // blocks with (i & size) == 0 sort best-first, the others reversed
          const bool first = (i & size) == 0;
          const bool jbetter = v[j] > v[i] || (v[j] == v[i] && id[j] < id[i]);
          if (first == jbetter) {
            const float tv = v[i]; v[i] = v[j]; v[j] = tv;
            const int ti = id[i]; id[i] = id[j]; id[j] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += 1024) out[i] = id[i];
}

// Visiting keys of a state under a ranking (the ranked search), without
// sorting: the ranking orders pixels by score, best first, ties by pixel
// id, and the search takes the first improving pixel of it, i.e. the
// improving pixel of highest score.  So per class ("sure": improving beyond
// its error band; "band": within it) one arg-max gives the pixel, and one
// count over the scores gives its position in the ranking (the number of
// pixels ranked before it), which is what the key and the attempt count
// need.  Scores: the FP32 ones of the mixed form unless the state is exact
// after an FP64 refresh; src 0 reads the FP64 scores P.df (plain, R-form).
// The search visits the ranking from its top: the state's cursor is reset.
// One workgroup of 1024 threads.
__device__ __forceinline__ bool rank_before(float sa, int a, float sb, int b) {
  return sa > sb || (sa == sb && a < b);
}

__global__ __launch_bounds__(1024) void k_ranked_keys(ProbDev P, const float* score,
                                                      DbsState* st, int src, uint32_t* key_sure,
                                                      uint32_t* key_band) {
  __shared__ float rs[2][16];
  __shared__ int ri[2][16];
  __shared__ int cnt[2][16];
  __shared__ float bs[2];
  __shared__ int bi[2];
  const int n = P.nd, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double f = st->f, eta = st->eta;
  const bool exact = src == 0 || st->exact;
  // best-ranked candidate of each class (-1: none)
  float s2[2] = {-INFINITY, -INFINITY};
  int i2[2] = {-1, -1};
  for (int i = tid; i < n; i += 1024) {
    const double df = exact ? P.df[i] : P.df32[i];
    const double margin = df - eta * f;
    int cls = -1;
    if (exact) {
      if (margin > 0.0) cls = 0;
    } else {
      const double band = P.band * P.dfb[i];
      if (margin > band) cls = 0;
      else if (margin >= -band) cls = 1;
    }
    if (cls >= 0 && (i2[cls] < 0 || rank_before(score[i], i, s2[cls], i2[cls]))) {
      s2[cls] = score[i];
      i2[cls] = i;
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float so = __shfl_xor(s2[c], o, 64);
      const int io = __shfl_xor(i2[c], o, 64);
      if (io >= 0 && (i2[c] < 0 || rank_before(so, io, s2[c], i2[c]))) {
        s2[c] = so;
        i2[c] = io;
      }
    }
    if (lane == 0) {
      rs[c][w] = s2[c];
      ri[c][w] = i2[c];
    }
  }
  __syncthreads();
  if (tid < 2) {
    float sb = -INFINITY;
    int ib = -1;
    for (int q = 0; q < 16; ++q)
      if (ri[tid][q] >= 0 && (ib < 0 || rank_before(rs[tid][q], ri[tid][q], sb, ib))) {
        sb = rs[tid][q];
        ib = ri[tid][q];
      }
    bs[tid] = sb;
    bi[tid] = ib;
  }
  __syncthreads();
  // positions: pixels ranked before each class's pick
  int c2[2] = {0, 0};
  for (int i = tid; i < n; i += 1024) {
    const float si = score[i];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      if (bi[c] >= 0 && rank_before(si, i, bs[c], bi[c])) c2[c] += 1;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c2[c] += __shfl_xor(c2[c], o, 64);
    if (lane == 0) cnt[c][w] = c2[c];
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t k[2];
    for (int c = 0; c < 2; ++c) {
      int tot = 0;
      for (int q = 0; q < 16; ++q) tot += cnt[c][q];
      k[c] = bi[c] >= 0 ? pack_key(tot, bi[c]) : kNoKey;
    }
    *key_sure = k[0];
    *key_band = k[1];
    st->cursor_s = 0;
    st->cursor_pos = 0;
  }
}

// ------------------------------------------------------------------ model
struct Model {
  int H = 0, W = 0, maxb = 0;
  int np = 0;                        // flat parameter count
  int off_w[kLayers], off_b[kLayers];
  int kpad[kLayers], ktpad[kLayers];
  std::vector<float> host_params;    // initial weights
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  int step = 0;
  std::string err;
  // device
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  short *wb[kLayers] = {}, *wt[kLayers] = {};
  float* X = nullptr;                // input [maxb][kCh[0]][H][W]
  float* T = nullptr;                // targets [maxb][1][H][W]
  float* Z[kLayers] = {};            // pre-activations
  float* dZ[2] = {};                 // gradient ping-pong
  float* gpart = nullptr;            // per-chunk partial weight gradients
  double* loss = nullptr;            // per-workgroup loss sums
};

constexpr int kWgradChunk = 256;     // pixels per partial weight gradient

}  // namespace pngf

struct pngf_model : pngf::Model {};

namespace {

thread_local std::string g_model_error;

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int mfail(pngf_model* m, int code, const std::string& msg) {
  if (m) m->err = msg; else g_model_error = msg;
  return code;
}

#define MCHK(m, call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return mfail(m, PNGF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Largest per-chunk partial gradient buffer over the layers (floats).
size_t gpart_floats(const pngf_model* m) {
  using namespace pngf;
  const size_t img = size_t(m->maxb) * m->H * m->W;
  const size_t nchunk = (img + kWgradChunk - 1) / kWgradChunk;
  size_t mx = 0;
  for (int l = 0; l < kLayers; ++l)
    mx = std::max(mx, size_t(kCh[l + 1]) * kCh[l] * 9 + kCh[l + 1]);
  return nchunk * mx;
}

size_t model_bytes(const pngf_model* m) {
  using namespace pngf;
  const size_t img = size_t(m->maxb) * m->H * m->W;
  size_t b = 4 * a256(size_t(m->np) * sizeof(float));
  for (int l = 0; l < kLayers; ++l)
    b += a256(size_t(pad16(kCh[l + 1])) * m->kpad[l] * 2) +
         a256(size_t(pad16(kCh[l])) * m->ktpad[l] * 2);
  b += a256(img * kCh[0] * sizeof(float)) + a256(img * sizeof(float));
  for (int l = 0; l < kLayers; ++l) b += a256(img * kCh[l + 1] * sizeof(float));
  b += 2 * a256(img * 32 * sizeof(float));
  b += a256(gpart_floats(m) * sizeof(float)) + a256(((img + 255) / 256) * sizeof(double));
  return b;
}

hipError_t pack_all(pngf_model* m) {
  using namespace pngf;
  for (int l = 0; l < kLayers; ++l) {
    const int cnt = kCh[l + 1] * kCh[l] * 9;
    hipLaunchKernelGGL(k_pack, dim3((cnt + 255) / 256), dim3(256), 0, m->stream,
                       m->w + m->off_w[l], kCh[l], kCh[l + 1], m->wb[l], m->kpad[l], m->wt[l],
                       m->ktpad[l]);
  }
  return hipGetLastError();
}

hipError_t conv_launch(pngf_model* m, const float* X, int Cin, int relu_in, const short* Wb,
                       int Kpad, const float* bias, float* Y, int Cout, int N, const float* gate) {
  using namespace pngf;
  const int waves = N * m->H * ((m->W + 15) / 16) * (pad16(Cout) / 16);
  hipLaunchKernelGGL(k_conv, dim3((waves + 3) / 4), dim3(256), 0, m->stream, X, Cin, relu_in,
                     Wb, Kpad, bias, Y, Cout, N, m->H, m->W, gate);
  return hipGetLastError();
}

// Forward pass on N images already in m->X; output in m->Z[3].
hipError_t forward(pngf_model* m, int N) {
  using namespace pngf;
  const float* in = m->X;
  for (int l = 0; l < kLayers; ++l) {
    hipError_t e = conv_launch(m, in, kCh[l], l > 0 ? 1 : 0, m->wb[l], m->kpad[l],
                               m->w + m->off_b[l], m->Z[l], kCh[l + 1], N, nullptr);
    if (e != hipSuccess) return e;
    in = m->Z[l];
  }
  return hipSuccess;
}

}  // namespace

namespace pngf {
// Internal interface used by the learned search in pngf_api.hip.
hipError_t model_score_state(pngf_model* m, const ProbDev& P, float** scores) {
  if (int64_t(m->H) * m->W != P.nd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_features, dim3(1), dim3(1024), 0, m->stream, P, m->H, m->W, m->X);
  hipError_t e = forward(m, 1);
  *scores = m->Z[kLayers - 1];
  return e;
}
hipError_t launch_rank(const float* s, int n, int32_t* out, hipStream_t st) {
  if (n < 1 || n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rank, dim3(1), dim3(1024), 0, st, s, n, out);
  return hipGetLastError();
}
int model_hw(pngf_model* m, int* H, int* W) {
  *H = m->H;
  *W = m->W;
  return m->bound ? PNGF_OK : PNGF_ESTATE;
}
hipStream_t model_stream(pngf_model* m) { return m->stream; }
hipError_t launch_ranked_keys(const ProbDev& P, const float* score, DbsState* st, int src,
                              uint32_t* key_sure, uint32_t* key_band, hipStream_t s) {
  if (P.nd < 1 || P.nd > kMaxPixels) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ranked_keys, dim3(1), dim3(1024), 0, s, P, score, st, src, key_sure,
                     key_band);
  return hipGetLastError();
}
hipError_t launch_features(const ProbDev& P, int H, int W, float* X, hipStream_t s) {
  if (int64_t(H) * W != P.nd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_features, dim3(1), dim3(1024), 0, s, P, H, W, X);
  return hipGetLastError();
}
}  // namespace pngf

extern "C" {

const char* pngf_model_last_error(const pngf_model* m) {
  return m ? m->err.c_str() : g_model_error.c_str();
}

int pngf_model_create(int32_t H, int32_t W, int32_t max_batch, uint64_t seed, pngf_model** out) {
  using namespace pngf;
  if (!out) return mfail(nullptr, PNGF_EINVAL, "null output pointer");
  *out = nullptr;
  if (H < 1 || W < 1 || max_batch < 1 || H * W > 8192)
    return mfail(nullptr, PNGF_EINVAL, "need 1 <= H*W <= 8192 and max_batch >= 1");
  pngf_model* m = new (std::nothrow) pngf_model();
  if (!m) return mfail(nullptr, PNGF_ENOMEM, "out of host memory");
  m->H = H;
  m->W = W;
  m->maxb = max_batch;
  int off = 0;
  for (int l = 0; l < kLayers; ++l) {
    m->off_w[l] = off;
    off += kCh[l + 1] * kCh[l] * 9;
    m->off_b[l] = off;
    off += kCh[l + 1];
    m->kpad[l] = pad16(kCh[l] * 9);
    m->ktpad[l] = pad16(kCh[l + 1] * 9);
  }
  m->np = off;
  m->host_params.assign(off, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 0; l < kLayers; ++l) {
    const double std = std::sqrt(2.0 / (kCh[l] * 9));   // He-normal
    for (int e = 0; e < kCh[l + 1] * kCh[l] * 9; ++e)
      m->host_params[m->off_w[l] + e] = float(nd(rng) * std);
  }
  *out = m;
  return PNGF_OK;
}

int pngf_model_num_params(pngf_model* m, int32_t* n) {
  if (!m || !n) return PNGF_EINVAL;
  *n = m->np;
  return PNGF_OK;
}

int pngf_model_workspace_bytes(pngf_model* m, size_t* bytes) {
  if (!m || !bytes) return PNGF_EINVAL;
  *bytes = model_bytes(m);
  return PNGF_OK;
}

int pngf_model_bind(pngf_model* m, void* dev_ws, size_t bytes, void* stream) {
  using namespace pngf;
  if (!m || !dev_ws) return PNGF_EINVAL;
  if (bytes < model_bytes(m)) return mfail(m, PNGF_ENOMEM, "model workspace too small");
  if (reinterpret_cast<uintptr_t>(dev_ws) & 255)
    return mfail(m, PNGF_EINVAL, "workspace must be 256-byte aligned");
  m->ws = static_cast<char*>(dev_ws);
  m->ws_bytes = bytes;
  m->stream = static_cast<hipStream_t>(stream);
  size_t off = 0;
  auto take = [&](size_t b) { char* p = m->ws + off; off += a256(b); return p; };
  const size_t img = size_t(m->maxb) * m->H * m->W;
  m->w = reinterpret_cast<float*>(take(size_t(m->np) * 4));
  m->g = reinterpret_cast<float*>(take(size_t(m->np) * 4));
  m->m = reinterpret_cast<float*>(take(size_t(m->np) * 4));
  m->v = reinterpret_cast<float*>(take(size_t(m->np) * 4));
  for (int l = 0; l < kLayers; ++l) {
    m->wb[l] = reinterpret_cast<short*>(take(size_t(pad16(kCh[l + 1])) * m->kpad[l] * 2));
    m->wt[l] = reinterpret_cast<short*>(take(size_t(pad16(kCh[l])) * m->ktpad[l] * 2));
  }
  m->X = reinterpret_cast<float*>(take(img * kCh[0] * 4));
  m->T = reinterpret_cast<float*>(take(img * 4));
  for (int l = 0; l < kLayers; ++l) m->Z[l] = reinterpret_cast<float*>(take(img * kCh[l + 1] * 4));
  m->dZ[0] = reinterpret_cast<float*>(take(img * 32 * 4));
  m->dZ[1] = reinterpret_cast<float*>(take(img * 32 * 4));
  m->gpart = reinterpret_cast<float*>(take(gpart_floats(m) * sizeof(float)));
  m->loss = reinterpret_cast<double*>(take(((img + 255) / 256) * sizeof(double)));
  MCHK(m, hipMemsetAsync(m->ws, 0, model_bytes(m), m->stream));
  MCHK(m, hipMemcpyAsync(m->w, m->host_params.data(), size_t(m->np) * 4, hipMemcpyHostToDevice,
                         m->stream));
  MCHK(m, pack_all(m));
  MCHK(m, hipStreamSynchronize(m->stream));
  m->bound = true;
  m->step = 0;
  return PNGF_OK;
}

int pngf_model_get_params(pngf_model* m, float* params, int32_t n) {
  if (!m || !params || n != m->np) return PNGF_EINVAL;
  if (!m->bound) {
    std::memcpy(params, m->host_params.data(), size_t(n) * 4);
    return PNGF_OK;
  }
  MCHK(m, hipMemcpyAsync(params, m->w, size_t(n) * 4, hipMemcpyDeviceToHost, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  return PNGF_OK;
}

int pngf_model_set_params(pngf_model* m, const float* params, int32_t n) {
  if (!m || !params || n != m->np) return PNGF_EINVAL;
  std::memcpy(m->host_params.data(), params, size_t(n) * 4);
  if (!m->bound) return PNGF_OK;
  MCHK(m, hipMemcpyAsync(m->w, params, size_t(n) * 4, hipMemcpyHostToDevice, m->stream));
  MCHK(m, pack_all(m));
  MCHK(m, hipStreamSynchronize(m->stream));
  return PNGF_OK;
}

int pngf_model_forward(pngf_model* m, const float* X, int32_t N, float* Y) {
  using namespace pngf;
  if (!m || !X || !Y) return PNGF_EINVAL;
  if (!m->bound) return mfail(m, PNGF_ESTATE, "model is not bound");
  if (N < 1 || N > m->maxb) return mfail(m, PNGF_EINVAL, "batch size out of range");
  const size_t img = size_t(N) * m->H * m->W;
  MCHK(m, hipMemcpyAsync(m->X, X, img * kCh[0] * 4, hipMemcpyHostToDevice, m->stream));
  MCHK(m, forward(m, N));
  MCHK(m, hipMemcpyAsync(Y, m->Z[kLayers - 1], img * 4, hipMemcpyDeviceToHost, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  return PNGF_OK;
}

int pngf_model_train_step(pngf_model* m, const float* X, const float* T, int32_t N, float lr,
                          double* loss, float* grads) {
  using namespace pngf;
  if (!m || !X || !T) return PNGF_EINVAL;
  if (!m->bound) return mfail(m, PNGF_ESTATE, "model is not bound");
  if (N < 1 || N > m->maxb) return mfail(m, PNGF_EINVAL, "batch size out of range");
  const int HW = m->H * m->W;
  const size_t img = size_t(N) * HW;
  MCHK(m, hipMemcpyAsync(m->X, X, img * kCh[0] * 4, hipMemcpyHostToDevice, m->stream));
  MCHK(m, hipMemcpyAsync(m->T, T, img * 4, hipMemcpyHostToDevice, m->stream));
  MCHK(m, forward(m, N));
  float* d = m->dZ[0];
  const int nblk = int((img + 255) / 256);
  hipLaunchKernelGGL(k_huber, dim3(nblk), dim3(256), 0, m->stream,
                     m->Z[kLayers - 1], m->T, d, int(img), 1.f / float(img), m->loss);
  MCHK(m, hipGetLastError());
  const int chunk = kWgradChunk;
  const int nchunk = int((img + chunk - 1) / chunk);
  for (int l = kLayers - 1; l >= 0; --l) {
    const float* in = l > 0 ? m->Z[l - 1] : m->X;
    const int cin = kCh[l], cout = kCh[l + 1];
    const int waves = (pad16(cout) / 16) * (m->kpad[l] / 16) * nchunk;
    hipLaunchKernelGGL(k_wgrad, dim3((waves + 3) / 4), dim3(256), 0, m->stream, d, in, cin,
                       l > 0 ? 1 : 0, cout, N, m->H, m->W, m->gpart, m->kpad[l], chunk);
    MCHK(m, hipGetLastError());
    // weights then biases of layer l are adjacent in the flat parameters
    const int nl = cout * cin * 9 + cout;
    hipLaunchKernelGGL(k_wsum, dim3((nl + 255) / 256), dim3(256), 0, m->stream, m->gpart, nl,
                       nchunk, m->g + m->off_w[l]);
    MCHK(m, hipGetLastError());
    if (l > 0) {
      float* dn = (d == m->dZ[0]) ? m->dZ[1] : m->dZ[0];
      // dA_{l-1} = conv(dZ_l, flipped W_l); dZ_{l-1} = dA_{l-1} * (Z_{l-1} > 0)
      MCHK(m, conv_launch(m, d, cout, 0, m->wt[l], m->ktpad[l], nullptr, dn, cin, N,
                          m->Z[l - 1]));
      d = dn;
    }
  }
  if (grads) {
    MCHK(m, hipMemcpyAsync(grads, m->g, size_t(m->np) * 4, hipMemcpyDeviceToHost, m->stream));
  }
  if (lr > 0.f) {
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, float(m->step)), c2 = 1.f - std::pow(b2, float(m->step));
    hipLaunchKernelGGL(k_adam, dim3((m->np + 255) / 256), dim3(256), 0, m->stream, m->w, m->g,
                       m->m, m->v, m->np, lr, b1, b2, 1e-8f, c1, c2);
    MCHK(m, hipGetLastError());
    MCHK(m, pack_all(m));
  }
  std::vector<double> lpart(nblk);
  MCHK(m, hipMemcpyAsync(lpart.data(), m->loss, size_t(nblk) * sizeof(double),
                         hipMemcpyDeviceToHost, m->stream));
  MCHK(m, hipStreamSynchronize(m->stream));
  double lsum = 0.0;
  for (double v : lpart) lsum += v;
  if (loss) *loss = lsum / double(img);
  return PNGF_OK;
}

int pngf_model_destroy(pngf_model* m) {
  delete m;
  return PNGF_OK;
}

}  // extern "C"

// ------------------------------------------------- allocation-free forward
//
// Scratch of pngf_model_forward_noalloc in a file-scope device array (one
// copy per GPU, held until the process ends): the BF16 weights of the four
// layers (zero-padded to 16-multiples), then two activation buffers of
// kNoAllocMaxPixels x 32 floats.  Host code uses only the per-device address
// from hipGetSymbolAddress, never the array's name.
namespace {
constexpr int kNoAllocMaxPixels = 16384;                 // N * H * W per call
constexpr size_t kNoAllocWeightBytes = size_t(64) << 10;
constexpr size_t kNoAllocActFloats = size_t(kNoAllocMaxPixels) * 32;
constexpr size_t kNoAllocScratchBytes =
    kNoAllocWeightBytes + 2 * kNoAllocActFloats * sizeof(float);   // 4 MiB + 64 KiB
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up once
// per device, with that device current).
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

extern "C" int pngf_model_forward_noalloc(const float* params, int32_t n_params, const float* X,
                                          int32_t N, int32_t H, int32_t W, float* Y,
                                          void* stream) {
  using namespace pngf;
  if (!params || !X || !Y) return mfail(nullptr, PNGF_EINVAL, "null device pointer");
  if (N < 1 || H < 1 || W < 1)
    return mfail(nullptr, PNGF_EINVAL, "need N, H, W >= 1");
  if (int64_t(N) * H * W > kNoAllocMaxPixels)
    return mfail(nullptr, PNGF_EINVAL,
                 "N*H*W exceeds the allocation-free forward's limit of 16384 pixels");
  int off_w[kLayers], off_b[kLayers], kpad[kLayers], np = 0;
  size_t wb_off[kLayers], wb_end = 0;
  for (int l = 0; l < kLayers; ++l) {
    off_w[l] = np;
    np += kCh[l + 1] * kCh[l] * 9;
    off_b[l] = np;
    np += kCh[l + 1];
    kpad[l] = pad16(kCh[l] * 9);
    wb_off[l] = wb_end;
    wb_end += a256(size_t(pad16(kCh[l + 1])) * kpad[l] * sizeof(short));
  }
  if (n_params != np) return mfail(nullptr, PNGF_EINVAL, "n_params does not match the network");
  if (wb_end > kNoAllocWeightBytes) return mfail(nullptr, PNGF_EINVAL, "weights exceed scratch");
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess)
    return mfail(nullptr, PNGF_EDEVICE,
                 std::string("scratch address (hipGetSymbolAddress): ") + hipGetErrorString(e));
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* sp = static_cast<char*>(base);
  short* wb[kLayers];
  for (int l = 0; l < kLayers; ++l) wb[l] = reinterpret_cast<short*>(sp + wb_off[l]);
  float* act[2] = {reinterpret_cast<float*>(sp + kNoAllocWeightBytes),
                   reinterpret_cast<float*>(sp + kNoAllocWeightBytes) + kNoAllocActFloats};
  // the padded rows and columns of the packed weights must read as zero:
  // clear the weight region, then pack
  const int words = int(wb_end / 4);
  hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(sp), words);
  for (int l = 0; l < kLayers; ++l) {
    const int cnt = kCh[l + 1] * kCh[l] * 9;
    hipLaunchKernelGGL(k_pack, dim3((cnt + 255) / 256), dim3(256), 0, st, params + off_w[l],
                       kCh[l], kCh[l + 1], wb[l], kpad[l], static_cast<short*>(nullptr), 0);
  }
  // X -> act0 -> act1 -> act0 -> Y (ReLU applied on read by the next layer)
  const float* in = X;
  for (int l = 0; l < kLayers; ++l) {
    float* out = (l == kLayers - 1) ? Y : act[l & 1];
    const int waves = N * H * ((W + 15) / 16) * (pad16(kCh[l + 1]) / 16);
    hipLaunchKernelGGL(k_conv, dim3((waves + 3) / 4), dim3(256), 0, st, in, kCh[l],
                       l > 0 ? 1 : 0, wb[l], kpad[l], params + off_b[l], out, kCh[l + 1], N, H,
                       W, static_cast<const float*>(nullptr));
    in = out;
  }
  e = hipGetLastError();
  if (e != hipSuccess)
    return mfail(nullptr, PNGF_EDEVICE, std::string("forward launch: ") + hipGetErrorString(e));
  return PNGF_OK;
}
