// Launchers of the FP32 matrix-core inner steps (dense X stored in FP32 or BF16).
//
// Each product with X runs on v_mfma_f32_16x16x4f32 with FP32 accumulation;
// the waves' partial results are added in FP64.  The FP64 step difference Dl
// (tile-major, as on the FP64 path) is the master; its FP32 copy D32 and the
// FP32 C32 feed the matrix cores.  The full-gradient passes stay FP64.
//
// FP32 copies, in 1 KB tiles: for each 16-row block of d (D32) or 16-sample
// block (C32) and each 16-column slice, element (k, j) at float
// ((k / 16) (PC / 16) + j / 16) 256 + (((k % 16) / 4) 16 + j % 16) 4 + k % 4.
// D32 holds pad16(d) x PC floats; rows past d and columns past p must hold
// zeros.  PC is pad16(p).  The sample dot splits the rows of X into KS ranges
// (KS = 2 while pad16(b) / 16 < 256, so that the workgroups cover the compute
// units, else 1) and writes one partial C32 per range, partial z at
// C32 + z pad16(b) PC; the update adds the partials in FP32 when it loads them.
// C32 therefore holds 2 pad16(b) x PC floats; step_dot_f32 writes the rows
// past b as zeros.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lr {

// Partial z: C32_z[s, j] = fl32(scale_s sum_{r in range z} X[r, idx[s]] D32[r, j]),
// s < pad16(b), j < PC.
hipError_t step_dot_f32(const XView& X, int p, int64_t b, const int32_t* idx,
                        const double* scale, const float* D32, float* C32, int PC,
                        hipStream_t st, const Probe& pr = Probe());

// Dl <- Dl - eta (G + lam Dl - U), U[r, j] = sum_s X[r, idx[s]] C[s, j] (C the sum of
// the partials), for r < d,
// j < p (Dl tile-major FP64, G column-major d x p), and D32 = fl32(Dl).  b <= 8192.
hipError_t step_update_f32(const XView& X, int p, int64_t b, const int32_t* idx, const float* C32,
                           int PC, const double* G, double* Dl, float* D32, double lam,
                           double eta, hipStream_t st, const Probe& pr = Probe());

}  // namespace lr
