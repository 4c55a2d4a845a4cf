// Launchers of the BF16 matrix-core inner steps (dense BF16 X only).
//
// The FP64 operands of a step (the difference block and the sampled products)
// are carried as two BF16 parts, hi = bf16(x) and lo = bf16(x - hi), so each
// product with X (exact in BF16) is two v_mfma_f32_16x16x32_bf16 chains with
// FP32 accumulation whose results are added in FP64.  The FP64 master copy of
// the difference block is what the solver keeps; the full-gradient passes stay
// FP64, so every epoch restarts from an exactly computed residual.
//
// Split layouts (BF16 bit patterns), in the matrix-core B-operand order: for
// each block of 32 k (rows of d for Dh/Dlo, samples for Ch/Cl) and each
// 16-column slice, a contiguous tile of 512 values in which lane l = 16 q + c
// holds k = 8 q .. 8 q + 7 of column c.  Element (k, j) sits at
// ((k / 32) (PC / 16) + j / 16) 512 + (((k % 32) / 8) 16 + j % 16) 8 + k % 8.
// Dh/Dlo hold ldD x PC values (ldD = pad32(d)), Ch/Cl ldC x PC (ldC >=
// pad32(b)); rows past d (samples past b) and columns past p must hold zeros.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lr {

int64_t pad_to(int64_t x, int64_t m);

// Ch/Cl[j, s] = split(scale_s sum_r X[r, idx[s]] (Dh + Dlo)[r, j]), s < b, j < PC.
hipError_t step_dot_bf16(const XView& X, int p, int64_t b, const int32_t* idx,
                         const double* scale, const uint16_t* Dh, const uint16_t* Dlo,
                         int64_t ldD, uint16_t* Ch, uint16_t* Cl, int64_t ldC, int PC,
                         hipStream_t st, const Probe& pr = Probe());

// Dl <- Dl - eta (G + lam Dl - U), U[r, j] = sum_s X[r, idx[s]] (Ch + Cl)[j, s],
// for r < d, j < p (Dl, G: FP64 column-major, ld d); then Dh/Dlo = split(Dl).
// b <= 8192.
hipError_t step_update_bf16(const XView& X, int p, int64_t b, const int32_t* idx,
                            const uint16_t* Ch, const uint16_t* Cl, int64_t ldC, int PC,
                            const double* G, double* Dl, uint16_t* Dh, uint16_t* Dlo, int64_t ldD,
                            double lam, double eta, hipStream_t st, const Probe& pr = Probe());

}  // namespace lr
