// gfx950 kernels of the path for compressed-column (CSC) X.  The paper lets X
// be sparse with per-pass cost nnz(X) (Section 1 footnote; Theorem
// "svrgSolve").  All arithmetic is FP64; stored values are widened on load.
//
// Layout choices: d x p iterates that are gathered by row id (the pass's W,
// the inner steps' difference and gradient) are kept row-major with a padded
// row of PC doubles, so the PC lanes that own one nonzero read one contiguous
// row.  X^T W is a per-column gather (deterministic); X T goes through a
// row-ordered copy of X built once per plan, with long rows cut into chunks
// whose partial sums are added in chunk order (deterministic, and no single
// heavy row serialises the pass).  The inner-step update scatters into the
// rows of its b sampled columns with FP64 atomics, the rows that occur most
// often summed per workgroup in LDS first: this is the one place whose
// rounding order depends on timing.
#include "sparse.h"

#include <hip/hip_ext.h>
#include <hipcub/hipcub.hpp>

#include <math.h>

namespace lr {
namespace {

constexpr int NT = 256;
constexpr int SB = 64;   // sampled columns per workgroup in the scatter

inline unsigned blocks(int64_t count) { return (unsigned)((count + NT - 1) / NT); }

__device__ __forceinline__ double ldv(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double ldv(const float* p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double ldv(const uint16_t* p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)p[i]) << 16);
}

__global__ __launch_bounds__(NT) void k_check_ptr(const int32_t* __restrict__ cp, int64_t n,
                                                  int64_t nnz, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i > n) return;
  const int64_t a = cp[i];
  bool ok = a >= 0 && a <= nnz;
  if (i == 0) ok = ok && a == 0;
  if (i == n) ok = ok && a == nnz;
  if (i < n) ok = ok && (int64_t)cp[i + 1] >= a;
  if (!ok) atomicOr(bad, 1);
}

__global__ __launch_bounds__(NT) void k_check_rows(const int32_t* __restrict__ cp,
                                                   const int32_t* __restrict__ ri, int64_t n,
                                                   int64_t d, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  int64_t prev = -1;
  bool ok = true;
  const int64_t k1 = cp[i + 1];
  for (int64_t k = cp[i]; k < k1; ++k) {
    const int64_t r = ri[k];
    ok = ok && r > prev && r < d;
    prev = r;
  }
  if (!ok) atomicOr(bad, 2);
}

// Row-order sum of squares with separate multiply and add roundings.
template <typename TX>
__global__ __launch_bounds__(NT) void k_csc_colnorm(const TX* __restrict__ v,
                                                    const int32_t* __restrict__ cp, int64_t n,
                                                    double* __restrict__ w,
                                                    int* __restrict__ bad) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  const int64_t k1 = cp[i + 1];
  for (int64_t k = cp[i]; k < k1; ++k) {
    const double x = ldv(v, k);
    const double sq = x * x;
    s = s + sq;
  }
  w[i] = s;
  if (!isfinite(s)) atomicOr(bad, 1);
}

__global__ __launch_bounds__(NT) void k_iota(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

// Column of stored entry `pos` (< nnz): the largest i with cp[i] <= pos.
__device__ __forceinline__ int64_t col_of(const int32_t* __restrict__ cp, int64_t n, int64_t pos) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((int64_t)cp[mid] <= pos)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename TX>
__global__ __launch_bounds__(NT) void k_csr_fill(const int32_t* __restrict__ pos_sorted,
                                                 const int32_t* __restrict__ cp, int64_t n,
                                                 const TX* __restrict__ v, int64_t nnz,
                                                 int32_t* __restrict__ col, TX* __restrict__ val) {
  const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (k >= nnz) return;
  const int64_t pos = pos_sorted[k];
  col[k] = (int32_t)col_of(cp, n, pos);
  val[k] = v[pos];
}

// row_ptr[r] = first sorted entry with row id >= r, r = 0..d.
__global__ __launch_bounds__(NT) void k_row_ptr(const uint32_t* __restrict__ keys, int64_t nnz,
                                                int64_t d, int32_t* __restrict__ row_ptr) {
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r > d) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < r)
      lo = mid + 1;
    else
      hi = mid;
  }
  row_ptr[r] = (int32_t)lo;
}

__global__ __launch_bounds__(NT) void k_cm_to_rm(const double* __restrict__ W, int64_t d,
                                                 int ncols, double* __restrict__ Wrm, int PC) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= d * PC) return;
  const int64_t r = e / PC;
  const int c = (int)(e % PC);
  Wrm[e] = c < ncols ? W[(int64_t)c * d + r] : 0.0;
}

__global__ __launch_bounds__(NT) void k_rm_to_cm(const double* __restrict__ Wrm, int64_t d,
                                                 int ncols, int PC, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= d * ncols) return;
  const int64_t c = e / d, r = e % d;
  W[e] = Wrm[r * PC + c];
}

// PC lanes per column (NT / PC columns per workgroup): lane c sums column c of
// the gathered rows in stored order.
template <typename TX, int PC, bool GATHER>
__global__ __launch_bounds__(NT) void k_csc_rows_dot(const TX* __restrict__ v,
                                                     const int32_t* __restrict__ cp,
                                                     const int32_t* __restrict__ ri,
                                                     int64_t ncols, const int32_t* __restrict__ idx,
                                                     const double* __restrict__ scale,
                                                     const double* __restrict__ Mrm,
                                                     double* __restrict__ out) {
  constexpr int NG = NT / PC;
  const int g = threadIdx.x / PC, c = threadIdx.x % PC;
  const int64_t j = (int64_t)blockIdx.x * NG + g;
  if (g >= NG || j >= ncols) return;
  const int64_t i = GATHER ? (int64_t)idx[j] : j;
  const int64_t k0 = cp[i], k1 = cp[i + 1];
  double s = 0.0;
#pragma unroll 4
  for (int64_t k = k0; k < k1; ++k) s += ldv(v, k) * Mrm[(int64_t)ri[k] * PC + c];
  out[j * PC + c] = GATHER ? scale[j] * s : s;
}

// Partial sum of one chunk of a row: NG groups of PC lanes stride the chunk,
// then the groups are added in group order.
template <typename TX, int PC>
__global__ __launch_bounds__(NT) void k_csr_chunk(const TX* __restrict__ val,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ chunk_beg,
                                                  const double* __restrict__ T,
                                                  double* __restrict__ part) {
  constexpr int NG = NT / PC;
  __shared__ double red[NG * PC];
  const int g = threadIdx.x / PC, c = threadIdx.x % PC;
  const int64_t ch = blockIdx.x;
  if (g < NG) {
    double s = 0.0;
    const int64_t e1 = chunk_beg[ch + 1];
#pragma unroll 4
    for (int64_t e = chunk_beg[ch] + g; e < e1; e += NG) s += ldv(val, e) * T[(int64_t)col[e] * PC + c];
    red[g * PC + c] = s;
  }
  __syncthreads();
  if (threadIdx.x < PC) {
    double t = 0.0;
    for (int q = 0; q < NG; ++q) t += red[q * PC + threadIdx.x];
    part[ch * PC + threadIdx.x] = t;
  }
}

// One workgroup per row: NG groups of PC lanes stride the row's chunks, then
// the groups are added in group order (heavy rows own hundreds of chunks).
template <int PC>
__global__ __launch_bounds__(NT) void k_csr_rows(const double* __restrict__ part,
                                                 const int32_t* __restrict__ row_chunk, int64_t d,
                                                 int p, double alpha,
                                                 const double* __restrict__ A, double beta,
                                                 const double* __restrict__ B, double gamma,
                                                 double* __restrict__ out) {
  constexpr int NG = NT / PC;
  __shared__ double red[NG * PC];
  const int g = threadIdx.x / PC, c = threadIdx.x % PC;
  const int64_t r = blockIdx.x;
  if (g < NG) {
    double s = 0.0;
    const int64_t c1 = row_chunk[r + 1];
    for (int64_t ch = row_chunk[r] + g; ch < c1; ch += NG) s += part[ch * PC + c];
    red[g * PC + c] = s;
  }
  __syncthreads();
  if (threadIdx.x < p) {
    double s = 0.0;
    for (int q = 0; q < NG; ++q) s += red[q * PC + threadIdx.x];
    const int64_t o = (int64_t)threadIdx.x * d + r;
    double y = alpha * s;
    if (A) y += beta * A[o];
    if (B) y += gamma * B[o];
    out[o] = y;
  }
}

__global__ __launch_bounds__(NT) void k_rm_decay(int64_t count, const double* __restrict__ Grm,
                                                 double* __restrict__ Dlrm, double lam,
                                                 double eta) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= count) return;
  const double x = Dlrm[e];
  Dlrm[e] = x - eta * (Grm[e] + lam * x);
}

template <typename TX, int PC>
__global__ __launch_bounds__(NT) void k_csc_scatter(const TX* __restrict__ v,
                                                    const int32_t* __restrict__ cp,
                                                    const int32_t* __restrict__ ri, int64_t b,
                                                    const int32_t* __restrict__ idx,
                                                    const double* __restrict__ C, int p,
                                                    const int32_t* __restrict__ head_slot,
                                                    const int32_t* __restrict__ head_row, int H,
                                                    double eta, double* __restrict__ Dlrm) {
  constexpr int NG = NT / PC, HCAP = 8192 / PC;
  __shared__ double acc[HCAP * PC];
  for (int e = threadIdx.x; e < H * PC; e += NT) acc[e] = 0.0;
  __syncthreads();
  const int g = threadIdx.x / PC, c = threadIdx.x % PC;
  if (g < NG && c < p) {
    const int64_t j0 = (int64_t)blockIdx.x * SB;
    const int64_t j1 = j0 + SB < b ? j0 + SB : b;
    for (int64_t j = j0 + g; j < j1; j += NG) {
      const int64_t i = idx[j];
      const double cj = eta * C[j * PC + c];
      const int64_t k1 = cp[i + 1];
      for (int64_t k = cp[i]; k < k1; ++k) {
        const int64_t r = ri[k];
        const double a = ldv(v, k) * cj;
        const int slot = head_slot[r];
        if (slot >= 0)
          atomicAdd(&acc[slot * PC + c], a);
        else
          unsafeAtomicAdd(&Dlrm[r * PC + c], a);
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < H * PC; e += NT) {
    const int c2 = e % PC;
    const double a = acc[e];
    if (c2 < p && a != 0.0) unsafeAtomicAdd(&Dlrm[(int64_t)head_row[e / PC] * PC + c2], a);
  }
}

}  // namespace

template <typename K, typename... A>
static void launch_sp(K kernel, dim3 grid, dim3 block, hipStream_t st, const Probe& pr,
                      A... args) {
  if (pr.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pr.start, pr.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

#define SP_DISPATCH_DT(dt, TX, ...) \
  switch (dt) {                     \
    case 0: {                       \
      using TX = double;            \
      __VA_ARGS__;                  \
    } break;                        \
    case 1: {                       \
      using TX = float;             \
      __VA_ARGS__;                  \
    } break;                        \
    case 2: {                       \
      using TX = uint16_t;          \
      __VA_ARGS__;                  \
    } break;                        \
    default:                        \
      return hipErrorInvalidValue;  \
  }

#define SP_DISPATCH_PC(PCv, PC, ...)  \
  switch (PCv) {                      \
    case 16: {                        \
      constexpr int PC = 16;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 32: {                        \
      constexpr int PC = 32;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 48: {                        \
      constexpr int PC = 48;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 64: {                        \
      constexpr int PC = 64;          \
      __VA_ARGS__;                    \
    } break;                          \
    default:                          \
      return hipErrorInvalidValue;    \
  }

hipError_t csc_check_ptr(const CscView& X, int* bad, hipStream_t st) {
  k_check_ptr<<<blocks(X.n + 1), NT, 0, st>>>(X.cp, X.n, X.nnz, bad);
  return hipGetLastError();
}

hipError_t csc_check_rows(const CscView& X, int* bad, hipStream_t st) {
  k_check_rows<<<blocks(X.n), NT, 0, st>>>(X.cp, X.ri, X.n, X.d, bad);
  return hipGetLastError();
}

hipError_t csc_colnorms(const CscView& X, double* w, int* bad, hipStream_t st) {
  SP_DISPATCH_DT(X.dt, TX,
                 k_csc_colnorm<TX><<<blocks(X.n), NT, 0, st>>>((const TX*)X.v, X.cp, X.n, w, bad));
  return hipGetLastError();
}

static int key_bits(int64_t d) {
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) < d) ++bits;
  return bits;
}

hipError_t csr_sort_bytes(int64_t nnz, int64_t d, size_t* bytes) {
  *bytes = 0;
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const uint32_t*)nullptr,
                                            (uint32_t*)nullptr, (const int32_t*)nullptr,
                                            (int32_t*)nullptr, (int)nnz, 0, key_bits(d));
}

hipError_t csr_build(const CscView& X, void* temp, size_t temp_bytes, uint32_t* keys_out,
                     int32_t* pos_in, int32_t* pos_out, int32_t* row_ptr, int32_t* col,
                     void* val, hipStream_t st) {
  if (X.nnz > 0) {
    k_iota<<<blocks(X.nnz), NT, 0, st>>>(pos_in, X.nnz);
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(
        temp, temp_bytes, (const uint32_t*)X.ri, keys_out, (const int32_t*)pos_in, pos_out,
        (int)X.nnz, 0, key_bits(X.d), st);
    if (e != hipSuccess) return e;
    SP_DISPATCH_DT(X.dt, TX,
                   k_csr_fill<TX><<<blocks(X.nnz), NT, 0, st>>>(pos_out, X.cp, X.n,
                                                                (const TX*)X.v, X.nnz, col,
                                                                (TX*)val));
  }
  k_row_ptr<<<blocks(X.d + 1), NT, 0, st>>>(keys_out, X.nnz, X.d, row_ptr);
  return hipGetLastError();
}

hipError_t cm_to_rm(const double* W, int64_t d, int ncols, double* Wrm, int PC, hipStream_t st) {
  if (ncols > PC) return hipErrorInvalidValue;
  k_cm_to_rm<<<blocks(d * PC), NT, 0, st>>>(W, d, ncols, Wrm, PC);
  return hipGetLastError();
}

hipError_t rm_to_cm(const double* Wrm, int64_t d, int ncols, int PC, double* W, hipStream_t st) {
  if (ncols > PC) return hipErrorInvalidValue;
  k_rm_to_cm<<<blocks(d * ncols), NT, 0, st>>>(Wrm, d, ncols, PC, W);
  return hipGetLastError();
}

hipError_t csc_xtw(const CscView& X, const double* Wrm, int PC, double* T, hipStream_t st,
                   const Probe& pr) {
  SP_DISPATCH_DT(X.dt, TX, SP_DISPATCH_PC(PC, PCT, {
    constexpr int NG = NT / PCT;
    launch_sp(k_csc_rows_dot<TX, PCT, false>, dim3((unsigned)((X.n + NG - 1) / NG)), dim3(NT), st,
              pr, (const TX*)X.v, X.cp, X.ri, X.n, (const int32_t*)nullptr,
              (const double*)nullptr, Wrm, T);
  }));
  return hipGetLastError();
}

hipError_t csr_xt(const CsrView& R, const double* T, int PC, int p, double* part, double alpha,
                  const double* A, double beta, const double* B, double gamma, double* out,
                  hipStream_t st, const Probe& pr) {
  if (p > PC) return hipErrorInvalidValue;
  if (R.nch > 0) {
    SP_DISPATCH_DT(R.dt, TX, SP_DISPATCH_PC(PC, PCT, {
      launch_sp(k_csr_chunk<TX, PCT>, dim3((unsigned)R.nch), dim3(NT), st, pr, (const TX*)R.val,
                R.col, R.chunk_beg, T, part);
    }));
  }
  SP_DISPATCH_PC(PC, PCT, {
    k_csr_rows<PCT><<<dim3((unsigned)R.d), NT, 0, st>>>(part, R.row_chunk, R.d, p, alpha, A, beta,
                                                        B, gamma, out);
  });
  return hipGetLastError();
}

hipError_t csc_step_dot(const CscView& X, int64_t b, const int32_t* idx, const double* scale,
                        const double* Dlrm, double* C, int PC, hipStream_t st, const Probe& pr) {
  SP_DISPATCH_DT(X.dt, TX, SP_DISPATCH_PC(PC, PCT, {
    constexpr int NG = NT / PCT;
    launch_sp(k_csc_rows_dot<TX, PCT, true>, dim3((unsigned)((b + NG - 1) / NG)), dim3(NT), st,
              pr, (const TX*)X.v, X.cp, X.ri, b, idx, scale, Dlrm, C);
  }));
  return hipGetLastError();
}

hipError_t rm_decay(int64_t count, const double* Grm, double* Dlrm, double lam, double eta,
                    hipStream_t st) {
  k_rm_decay<<<blocks(count), NT, 0, st>>>(count, Grm, Dlrm, lam, eta);
  return hipGetLastError();
}

int sp_head_cap(int PC) { return 8192 / PC; }

hipError_t csc_step_scatter(const CscView& X, int64_t b, const int32_t* idx, const double* C,
                            int PC, int p, const int32_t* head_slot, const int32_t* head_row,
                            int H, double eta, double* Dlrm, hipStream_t st, const Probe& pr) {
  if (H < 0 || H > sp_head_cap(PC) || p > PC) return hipErrorInvalidValue;
  SP_DISPATCH_DT(X.dt, TX, SP_DISPATCH_PC(PC, PCT, {
    launch_sp(k_csc_scatter<TX, PCT>, dim3((unsigned)((b + SB - 1) / SB)), dim3(NT), st, pr,
              (const TX*)X.v, X.cp, X.ri, b, idx, C, p, head_slot, head_row, H, eta, Dlrm);
  }));
  return hipGetLastError();
}

}  // namespace lr
