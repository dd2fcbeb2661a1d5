// Internal declarations shared by the host code and the HIP launchers of
// libpngf.  Not part of the C ABI.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pngf.h"

namespace pngf {

using cd = std::complex<double>;

// ---------------------------------------------------------------- host side
struct Grid {
  int nx = 0, ny = 0, npml = 0;
  double h = 0.0;
};

// Per-frequency precomputed data (host copies, FP64).
struct FreqData {
  double k0 = 0.0;
  double norm = 1.0;             // objective normalizer
  std::vector<cd> G;             // n_d x n_d row-major, symmetric
  std::vector<cd> b;             // n_d
  std::vector<cd> god;           // n_d (single output row)
  cd xb = 0.0;
};

struct Precomputed {
  Grid grid;
  int n_d = 0;
  double eps_lo = 1.0, eps_hi = 1.0;
  bool pec = false;                    // PEC pixels (pixel_kind PNGF_PIXEL_PEC)
  std::vector<int64_t> design_nodes;   // flat node ids of pixels, pixel order
  std::vector<FreqData> freq;
  double seconds = 0.0;
};

// Host precompute of one problem; returns PNGF_OK or an error code and fills
// err on failure.
int precompute(const pngf_problem* p, Precomputed* out, std::string* err);

// In-place FP64 inverse of a dense complex matrix (row-major, n x n, leading
// dimension ld) by Gauss-Jordan elimination with partial pivoting.  Returns
// PNGF_OK or PNGF_ESINGULAR.  Multithreaded with OpenMP.
int dense_inverse(cd* a, int n, int ld);

}  // namespace pngf
