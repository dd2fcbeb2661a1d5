// Device-side helpers shared by the libpngf HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pngf {

constexpr int kMaxFreq = 8;
constexpr int kRowThreads = 256;   // one workgroup streams one matrix row
constexpr int kMixRows = 8;        // rows per workgroup of the mixed step (two per wave)
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// Visiting keys: the place of a candidate in the visiting order (its
// position in the current sweep, or N_d + its position in the next sweep) in
// the high bits and the pixel in the low kKeyPixBits, so the minimum key
// names its pixel without a lookup.
constexpr int kKeyPixBits = 14;
constexpr uint32_t kKeyPixMask = (1u << kKeyPixBits) - 1u;
constexpr int kMaxPixels = 1 << kKeyPixBits;
__device__ __forceinline__ uint32_t pack_key(int vis, int pixel) {
  return (uint32_t(vis) << kKeyPixBits) | uint32_t(pixel);
}
__device__ __forceinline__ int key_vis(uint32_t k) { return int(k >> kKeyPixBits); }
__device__ __forceinline__ int key_pixel(uint32_t k) { return int(k & kKeyPixMask); }

struct z64 { double re, im; };
struct z32 { float re, im; };

__device__ __forceinline__ z64 zmul(z64 a, z64 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ z64 zsub(z64 a, z64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ z64 zscale(z64 a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ z64 zdiv(z64 a, z64 b) {
  double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ z64 zfma(z64 a, z64 b, z64 c) {  // a*b + c
  return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
__device__ __forceinline__ double zabs2(z64 a) { return a.re * a.re + a.im * a.im; }

// Broadcast of lane p's value to the wave (p wave-uniform).
__device__ __forceinline__ double lane_d(double v, int p) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b)), p));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(b >> 32)), p));
  return __longlong_as_double(static_cast<long long>((uint64_t(hi) << 32) | lo));
}

// Maximum over the wave: DPP exchanges within each row of 16 lanes (quad
// swaps, then rotations by 4 and 8), then the four row maxima by readlane.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  uint32_t o;
  o = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = o > v ? o : v;
  o = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = o > v ? o : v;
  o = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x124, 0xF, 0xF, false));  // row_ror 4
  v = o > v ? o : v;
  o = uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x128, 0xF, 0xF, false));  // row_ror 8
  v = o > v ? o : v;
  const uint32_t a = uint32_t(__builtin_amdgcn_readlane(int(v), 0));
  const uint32_t b = uint32_t(__builtin_amdgcn_readlane(int(v), 16));
  const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(v), 32));
  const uint32_t d = uint32_t(__builtin_amdgcn_readlane(int(v), 48));
  const uint32_t ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Sum over a full workgroup of kRowThreads lanes; result valid in every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup reduction of a complex double; `red` is LDS of >= 2*(threads/64)
// doubles.  Ends with a barrier so `red` may be reused.
__device__ __forceinline__ z64 block_zsum(z64 v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  if (lane == 0) { red[2 * wid] = v.re; red[2 * wid + 1] = v.im; }
  __syncthreads();
  z64 s{0.0, 0.0};
  for (int w = 0; w < nw; ++w) { s.re += red[2 * w]; s.im += red[2 * w + 1]; }
  __syncthreads();
  return s;
}

}  // namespace pngf
