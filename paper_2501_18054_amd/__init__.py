"""MI355X-native per-iteration hot path of the Precomputed Numerical Green
Function (PNGF) method: a C-ABI library (libpngf.so, HIP for gfx950) and its
thin ctypes binding."""
from .binding import (Handle, Batch, Model, PngfError, default_options, lib,
                      model_forward_noalloc, PNGF_FP64_PLAIN,
                      PNGF_MIXED, PNGF_RFORM, PNGF_FLAG_TIMING, PNGF_FLAG_STEP_LAUNCHES,
                      PNGF_FLAG_TIMING_STEPS, PNGF_FLAG_PIVOT_SEARCH,
                      PNGF_PIXEL_DIELECTRIC,
                      PNGF_PIXEL_PEC, EXPORTS, LIB_PATH)

__all__ = ["Handle", "Batch", "Model", "PngfError", "default_options", "lib",
           "model_forward_noalloc", "PNGF_FP64_PLAIN",
           "PNGF_MIXED", "PNGF_RFORM", "PNGF_FLAG_TIMING", "PNGF_FLAG_STEP_LAUNCHES",
           "PNGF_FLAG_TIMING_STEPS", "PNGF_FLAG_PIVOT_SEARCH",
           "PNGF_PIXEL_DIELECTRIC",
           "PNGF_PIXEL_PEC", "EXPORTS", "LIB_PATH"]
