// Matrix-core full-gradient pass for dense FP32 and BF16 X (gfx950
// v_mfma_f32_16x16x32_bf16): out = alpha X (X^T W) + beta A + gamma B.
//
// Operands are carried as sums of BF16 parts: W and T = X^T W as three parts
// (hi + mid + lo, 24 significant bits), FP32 X as three parts (an exact split),
// BF16 X as itself.  Products of parts whose indices add up to less than three
// are formed (six for FP32 X, three for BF16 X); matrix-core accumulation is
// FP32 and is added into FP64 every 256 terms of a contraction.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace lr {

// Workspace of one pass, all device memory; sizes from mc_sizes.
struct McBufs {
  uint16_t* Wp;     // W parts, 3 x wstride BF16 (matrix-core B-operand tiles)
  uint16_t* Tp;     // T parts, 3 x tstride BF16
  float* part;      // nsplit x d x PC FP32 partial sums of X T
  int64_t wstride, tstride;
  int nsplit;
};

struct McSizes {
  int64_t wp_elems, tp_elems, part_elems;   // BF16, BF16, FP32 element counts
  int nsplit;
};

// Sizes for X of d x n and PC = pad16(p) columns (p <= 64).
McSizes mc_sizes(int64_t d, int64_t n, int PC);

// X: dt 1 (FP32) or 2 (BF16), column-major with ld % 8 == 0 and a 16-byte
// aligned base (hipErrorInvalidValue otherwise).  W, A, B, out: d x p FP64
// column-major; A, B may be null.  pr times the X^T W kernel.
hipError_t mc_pass(const XView& X, const double* W, int p, int PC, const McBufs& mb,
                   double alpha, const double* A, double beta, const double* B, double gamma,
                   double* out, hipStream_t st, const Probe& pr = Probe(),
                   const Probe& pr2 = Probe());

}  // namespace lr
