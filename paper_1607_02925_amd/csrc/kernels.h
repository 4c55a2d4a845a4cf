// Launchers of the gfx950 kernels.  Every launcher enqueues on `st` and
// returns hipSuccess or the launch error.  Dense matrices are FP64
// column-major with leading dimension d unless stated otherwise; X is the
// caller's column-major matrix of dtype `dt` (0 f64, 1 f32, 2 bf16 bits).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lr {

// Optional start/stop events that time one kernel launch exactly.
struct Probe {
  hipEvent_t start = nullptr, stop = nullptr;
};

struct XView {
  const void* v;
  int64_t d, n, ld;
  int dt;
};

// Section 2.3 sampler table: w_i = ||x_i||^2 (row-order FP64 sums), NaN/Inf flag.
hipError_t colnorms(const XView& X, double* w, int* bad, hipStream_t st);
// wmax / sum(w) partials -> q_i -> cumulative table cdf[0..n] (uint64).
// scratch: >= 4 * nblocks(n) doubles.  fro2: device double.
hipError_t build_table(const double* w, int64_t n, uint64_t* cdf, double* fro2, double* scratch,
                       hipStream_t st);

// S (d x p) Gaussian block from Philox stream (tag, solve).
hipError_t gaussian(double* S, int64_t d, int p, uint64_t seed, uint32_t word3, hipStream_t st);

// Pass: T = X^T W (n x PC row-major, PC = pad16(p), padded columns zero), then
// out = alpha * X T + beta * A + gamma * B  (A, B may be null; d x p).
struct PassBufs {
  double* Ypart;   // nsplit * d * p partial sums
  int nsplit;
};
int pad16(int p);
int pass_nsplit(int64_t d, int64_t n);
// Wtile: scratch of pad16(d) x pad16(p) doubles (W in the tile-major form, see
// tile_add below).
hipError_t pass_xtw(const XView& X, const double* W, int p, double* T, int PC, double* Wtile,
                    hipStream_t st, const Probe& pr = Probe());
hipError_t pass_xt(const XView& X, const double* T, int PC, int p, const PassBufs& pb,
                   double alpha, const double* A, double beta, const double* B, double gamma,
                   double* out, hipStream_t st, const Probe& pr = Probe());

// Column draws of `steps` inner steps starting at step t0 of one epoch:
// idx/scale[(t - t0) * b + j].
hipError_t draw_chunk(int64_t n, const uint64_t* cdf, uint64_t seed, uint32_t t0, int64_t steps,
                      uint32_t epoch, uint32_t word3, int64_t b, int32_t* idx, double* scale,
                      hipStream_t st);
// The inner-step difference Dl of the dense FP64 path is kept tile-major: for
// each 16-row block blk and 16-column slice u a contiguous tile of 256 doubles
// at (blk * PC / 16 + u) * 256, element (row 4 q + s, column 16 u + c) of the
// block at (s / 2) * 128 + (16 q + c) * 2 + s % 2 -- lane 16 q + c of the FP64
// matrix-core B operand reads its four values with two 16-byte loads, and a
// wave reads the tile as two contiguous 1 KB pieces.  pad16(d) x PC doubles;
// rows >= d and columns >= p stay 0.
// out = W + Dl for the d x p column-major W (out may be W).
hipError_t tile_add(int64_t d, int p, int PC, const double* W, const double* Dl, double* out,
                    hipStream_t st);
// Inner step, part 1: C = diag(scale) X_B^T Dl   (C: b x PC row-major, Dl
// tile-major).  C must hold pad16(b) rows: rows b .. pad16(b) - 1 are set to 0.
hipError_t step_dot(const XView& X, int p, int64_t b, const int32_t* idx, const double* scale,
                    const double* Dl, double* C, int PC, hipStream_t st,
                    const Probe& pr = Probe());
// Deflation of an inner step (Section 3.1): with ns > 0 the update uses the
// sampled columns of (I - Ud Ud^T) X.  Z = X^T Ud (n x PCZ row-major, PCZ =
// pad16(ns)); Ud d x ns column-major (ld d); Vp scratch of nks x PCZ x PC
// doubles, nks = zbc_chunks(b).
struct Deflation {
  int ns = 0, PCZ = 0, nks = 0;
  const double* Z = nullptr;
  const double* Ud = nullptr;
  double* Vp = nullptr;
};
int zbc_chunks(int64_t b);
// Inner step, part 2: Dl <- Dl - eta (G + lam Dl - P X_B C), P = I - Ud Ud^T
// when deflating (else identity).  b <= 8192; Dl tile-major, G d x p column-major;
// C as written by step_dot (pad16(b) rows, zero past b).
hipError_t step_update(const XView& X, int p, int64_t b, const int32_t* idx, const double* C,
                       int PC, const double* G, double* Dl, double lam, double eta,
                       hipStream_t st, const Probe& pr = Probe(),
                       const Deflation& df = Deflation());
// Draw only (for testing the sampler).
hipError_t sample_only(int64_t n, const uint64_t* cdf, uint64_t seed, uint32_t step,
                       uint32_t epoch, uint32_t word3, int64_t b, int32_t* idx, double* scale,
                       hipStream_t st);

// G = A^T B  (A: rows x pa, B: rows x pb, arbitrary row/col strides), FP64,
// deterministic two-stage reduction.  part: >= gram_nblk(rows) * pa * pb.
int gram_nblk(int64_t rows);
hipError_t gram(const double* A, int64_t rsa, int64_t csa, int pa, const double* B, int64_t rsb,
                int64_t csb, int pb, int64_t rows, double* part, double* G, hipStream_t st);
// sum of squares of `count` elements -> out[0] (deterministic); part >= 1024.
hipError_t sumsq(const double* A, int64_t count, double* part, double* out, hipStream_t st);

// D (d x q) = A (d x p) M (p x q, ld ldm) + beta C.
hipError_t gemm_small(int64_t d, int p, int q, const double* A, const double* M, int ldm, double* D,
                      double beta, const double* C, hipStream_t st);
// out = a*X + b*Y + c*Z elementwise (Y, Z may be null).
hipError_t lincomb(int64_t count, double a, const double* X, double b, const double* Y, double c,
                   const double* Z, double* out, hipStream_t st);

// Single-workgroup small dense kernels (m <= 64).
// Cholesky of G (m x m, symmetrised), Rinv = R^{-1} (R = L^T upper); info = 1 if not SPD.
hipError_t chol_rinv(const double* G, int m, double* Rinv, int* info, hipStream_t st);
// Jacobi eigendecomposition, descending, sign-fixed eigenvectors (m x m col-major).
hipError_t eigh(const double* H, int m, double* vals, double* vecs, hipStream_t st);
// M = Q diag(1 / (lam - vals)) Q^T.
hipError_t shift_inverse(const double* vals, const double* Q, int m, double lam, double* M,
                         hipStream_t st);
// out[i] = || A[:, i] - theta_i B[:, i] ||  for i < m   (A, B: d x m).
hipError_t residual_norms(const double* A, const double* B, const double* theta, int64_t d, int m,
                          double* out, hipStream_t st);
// Make each column's largest-magnitude entry positive (first index on ties).
hipError_t sign_fix(double* U, int64_t d, int k, hipStream_t st);
// Every byte of [p, p + bytes) set to `byte` by a kernel (p 4-byte aligned).
hipError_t fill_bytes(void* p, size_t bytes, unsigned char byte, hipStream_t st);

}  // namespace lr
