// gfx950 kernels of the shift-and-invert low-rank path.  All arithmetic is
// FP64; X is read in its storage type (f64, f32 or bf16 bit patterns) and
// widened on load.  See kernels.h for the contract of each launcher.
#include "kernels.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace lr {
namespace {

constexpr int NT = 256;  // threads per workgroup for the streaming kernels

__device__ __forceinline__ double ldx(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double ldx(const float* p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double ldx(const uint16_t* p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)p[i]) << 16);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox-4x32
// bijection, key bumped by the Weyl constants between rounds.
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 o;
    o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    o.y = (uint32_t)p1;
    o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    o.w = (uint32_t)p0;
    c = o;
  }
  return c;
}

// Largest i in [0, n) with cdf[i] <= r, for r < cdf[n].
__device__ __forceinline__ int64_t cdf_search(const uint64_t* __restrict__ cdf, int64_t n,
                                              uint64_t r) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (cdf[mid] <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One draw of the column sampler: counter (j, step, epoch, word3).
__device__ __forceinline__ void draw_one(const uint64_t* __restrict__ cdf, int64_t n, uint32_t k0,
                                         uint32_t k1, uint32_t j, uint32_t step, uint32_t epoch,
                                         uint32_t word3, int64_t b, int64_t* idx, double* scale) {
  const U4 o = philox10({j, step, epoch, word3}, k0, k1);
  const uint64_t u = ((uint64_t)o.x << 32) | (uint64_t)o.y;
  const uint64_t Q = cdf[n];
  const uint64_t r = __umul64hi(u, Q);
  const int64_t i = cdf_search(cdf, n, r);
  const uint64_t q = cdf[i + 1] - cdf[i];
  *idx = i;
  *scale = (double)Q / ((double)b * (double)q);
}

// ---------------------------------------------------------------------------
// Column squared norms, summed in row order with separate multiply and add
// roundings (no fused multiply-add), so every implementation agrees bit for bit.
// A workgroup owns CN_COLS columns and walks down them CN_ROWS rows at a
// time: the tile is loaded with consecutive threads on consecutive rows of a
// column (coalesced), then each of CN_COLS threads adds its column's values
// from LDS in row order.
constexpr int CN_COLS = 64, CN_ROWS = 64;
template <typename TX>
__global__ __launch_bounds__(NT) void k_colnorm(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                int64_t n, double* __restrict__ w,
                                                int* __restrict__ bad) {
#pragma clang fp contract(off)
  __shared__ double tile[CN_COLS][CN_ROWS + 1];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * CN_COLS;
  double s = 0.0;
  for (int64_t r0 = 0; r0 < d; r0 += CN_ROWS) {
    for (int e = t; e < CN_COLS * CN_ROWS; e += NT) {
      const int c = e / CN_ROWS, r = e % CN_ROWS;
      tile[c][r] = (c0 + c < n && r0 + r < d) ? ldx(X + (c0 + c) * ld, r0 + r) : 0.0;
    }
    __syncthreads();
    if (t < CN_COLS) {
      const int rn = (int)min<int64_t>(CN_ROWS, d - r0);
      for (int r = 0; r < rn; ++r) {
        const double x = tile[t][r];
        const double sq = x * x;
        s = s + sq;
      }
    }
    __syncthreads();
  }
  if (t < CN_COLS && c0 + t < n) {
    w[c0 + t] = s;
    if (!isfinite(s)) atomicOr(bad, 1);
  }
}

constexpr int TB = 1024;  // table elements per block (4 per thread)

__global__ __launch_bounds__(NT) void k_wstats(const double* __restrict__ w, int64_t n,
                                               double* __restrict__ pmax,
                                               double* __restrict__ psum) {
  __shared__ double smax[NT], ssum[NT];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * TB;
  double mx = 0.0, sm = 0.0;
  for (int e = 0; e < TB / NT; ++e) {
    const int64_t i = base + e * NT + t;
    if (i < n) {
      const double v = w[i];
      mx = fmax(mx, v);
      sm += v;
    }
  }
  smax[t] = mx;
  ssum[t] = sm;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      smax[t] = fmax(smax[t], smax[t + s]);
      ssum[t] += ssum[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    pmax[blockIdx.x] = smax[0];
    psum[blockIdx.x] = ssum[0];
  }
}

// Reduces the per-block partials in a fixed order: out[0] = max, out[1] = sum.
__global__ __launch_bounds__(NT) void k_wfinal(const double* __restrict__ pmax,
                                               const double* __restrict__ psum, int64_t nb,
                                               double* __restrict__ out,
                                               double* __restrict__ fro2) {
  __shared__ double smax[NT], ssum[NT];
  const int t = threadIdx.x;
  double mx = 0.0, sm = 0.0;
  for (int64_t b = t; b < nb; b += NT) {
    mx = fmax(mx, pmax[b]);
    sm += psum[b];
  }
  smax[t] = mx;
  ssum[t] = sm;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      smax[t] = fmax(smax[t], smax[t + s]);
      ssum[t] += ssum[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = smax[0];
    out[1] = ssum[0];
    *fro2 = ssum[0];
  }
}

// q_i = floor(2^24 w_i / wmax) + 1 (0 for w_i = 0), written to cdf[i+1];
// per-block sums to bsum.
__global__ __launch_bounds__(NT) void k_quant(const double* __restrict__ w, int64_t n,
                                              const double* __restrict__ stats,
                                              uint64_t* __restrict__ cdf,
                                              uint64_t* __restrict__ bsum) {
  __shared__ uint64_t ss[NT];
  const int t = threadIdx.x;
  const double wmax = stats[0];
  const int64_t base = (int64_t)blockIdx.x * TB;
  uint64_t acc = 0;
  for (int e = 0; e < TB / NT; ++e) {
    const int64_t i = base + e * NT + t;
    if (i < n) {
      const double v = w[i];
      const uint64_t q = v > 0.0 ? (uint64_t)floor((v / wmax) * 16777216.0) + 1ull : 0ull;
      cdf[i + 1] = q;
      acc += q;
    }
  }
  ss[t] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) ss[t] += ss[t + s];
    __syncthreads();
  }
  if (t == 0) bsum[blockIdx.x] = ss[0];
}

// In-place exclusive scan of bsum[0..nb) by one workgroup.
__global__ __launch_bounds__(NT) void k_scan_bsum(uint64_t* __restrict__ bsum, int64_t nb) {
  __shared__ uint64_t s[NT];
  __shared__ uint64_t carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += NT) {
    const int64_t i = c0 + t;
    const uint64_t v = i < nb ? bsum[i] : 0;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
      const uint64_t add = t >= off ? s[t - off] : 0;
      __syncthreads();
      s[t] += add;
      __syncthreads();
    }
    const uint64_t incl = s[t];
    const uint64_t base = carry;
    __syncthreads();
    if (i < nb) bsum[i] = base + incl - v;
    if (t == NT - 1) carry = base + incl;
    __syncthreads();
  }
}

// cdf[i+1] = boff[block] + inclusive scan of q within the block; cdf[0] = 0.
__global__ __launch_bounds__(NT) void k_scan_local(uint64_t* __restrict__ cdf, int64_t n,
                                                   const uint64_t* __restrict__ boff) {
  __shared__ uint64_t s[NT];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * TB + (int64_t)t * (TB / NT);
  uint64_t v[TB / NT];
  uint64_t run = 0;
  for (int e = 0; e < TB / NT; ++e) {
    const int64_t i = base + e;
    v[e] = i < n ? cdf[i + 1] : 0;
    run += v[e];
  }
  s[t] = run;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const uint64_t add = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  uint64_t pre = boff[blockIdx.x] + s[t] - run;
  for (int e = 0; e < TB / NT; ++e) {
    const int64_t i = base + e;
    pre += v[e];
    if (i < n) cdf[i + 1] = pre;
  }
  if (blockIdx.x == 0 && t == 0) cdf[0] = 0;
}

// ---------------------------------------------------------------------------
// Gaussian block: element (i, j) from counter (i, j, 0, word3), Box-Muller.
__global__ __launch_bounds__(NT) void k_gauss(double* __restrict__ S, int64_t d, int p,
                                              uint32_t k0, uint32_t k1, uint32_t word3) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= d * p) return;
  const int64_t i = e % d;
  const int64_t j = e / d;
  const U4 o = philox10({(uint32_t)i, (uint32_t)j, 0u, word3}, k0, k1);
  const double u1 = ((double)(((uint64_t)o.x << 21) | (uint64_t)(o.y >> 11)) + 0.5) * 0x1p-53;
  const double u2 = ((double)(((uint64_t)o.z << 21) | (uint64_t)(o.w >> 11)) + 0.5) * 0x1p-53;
  S[e] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// ---------------------------------------------------------------------------
// FP64 matrix-core tiles.  v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; its result register v holds D[4*v + l/16][l%16].
// The K index is permuted so that, over four consecutive instructions
// s = 0..3, lane l covers K positions 4*(l/16)+s: four consecutive rows of one
// column, which one vector load fetches.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// v_mfma_f64_4x4x4f64, four 4 x 4 blocks: lane l = 16 k + 4 blk + m supplies
// A[blk][m][k] and lane 16 k + 4 blk + n supplies B[blk][k][n]; lane
// 16 m + 4 blk + n receives D[blk][m][n] (checked on the device).  With the
// 16x16x4 A operand in place (lane l: row l % 16, k = l / 16) the four blocks
// cover the same 16 rows against four columns of B, at a quarter of the
// 16x16x4 cost (16 against 64 cycles per SIMD, measured).
__device__ __forceinline__ double mfma_f64_4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive elements X[r..r+3] of one column, widened to FP64.  VEC:
// the column base and r are aligned for one vector load; rows >= d read 0.
template <typename TX, bool VEC>
__device__ __forceinline__ void load4(const TX* __restrict__ col, int64_t r, int64_t d,
                                      double* x) {
  if (VEC && r + 3 < d) {
    if constexpr (sizeof(TX) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(col + r);
      const double2 b = *reinterpret_cast<const double2*>(col + r + 2);
      x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
    } else if constexpr (sizeof(TX) == 4) {
      const float4 a = *reinterpret_cast<const float4*>(col + r);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    } else {
      const uint2 a = *reinterpret_cast<const uint2*>(col + r);
      x[0] = (double)__uint_as_float(a.x << 16);
      x[1] = (double)__uint_as_float(a.x & 0xFFFF0000u);
      x[2] = (double)__uint_as_float(a.y << 16);
      x[3] = (double)__uint_as_float(a.y & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) x[s] = (r + s < d) ? ldx(col, r + s) : 0.0;
  }
}

// Four consecutive column elements kept in the storage type until use, so
// that a prefetch group costs 4 (f32), 2 (bf16) or 8 (f64) registers.
template <typename TX>
struct Raw4;
template <>
struct Raw4<double> {
  double v[4];
  __device__ __forceinline__ double get(int s) const { return v[s]; }
  __device__ __forceinline__ void zero() { v[0] = v[1] = v[2] = v[3] = 0.0; }
};
template <>
struct Raw4<float> {
  float v[4];
  __device__ __forceinline__ double get(int s) const { return (double)v[s]; }
  __device__ __forceinline__ void zero() { v[0] = v[1] = v[2] = v[3] = 0.0f; }
};
template <>
struct Raw4<uint16_t> {
  uint32_t w[2];  // element 2i in the low half of w[i], 2i+1 in the high half
  __device__ __forceinline__ double get(int s) const {
    const uint32_t x = w[s >> 1];
    return (double)__uint_as_float((s & 1) ? (x & 0xFFFF0000u) : (x << 16));
  }
  __device__ __forceinline__ void zero() { w[0] = w[1] = 0u; }
};

template <typename TX, bool VEC>
__device__ __forceinline__ void load4raw(const TX* __restrict__ col, int64_t r, int64_t d,
                                         Raw4<TX>& o) {
  if (VEC && r + 3 < d) {
    if constexpr (sizeof(TX) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(col + r);
      const double2 b = *reinterpret_cast<const double2*>(col + r + 2);
      o.v[0] = a.x; o.v[1] = a.y; o.v[2] = b.x; o.v[3] = b.y;
    } else if constexpr (sizeof(TX) == 4) {
      const float4 a = *reinterpret_cast<const float4*>(col + r);
      o.v[0] = a.x; o.v[1] = a.y; o.v[2] = a.z; o.v[3] = a.w;
    } else {
      const uint2 a = *reinterpret_cast<const uint2*>(col + r);
      o.w[0] = a.x; o.w[1] = a.y;
    }
  } else {
    if constexpr (sizeof(TX) == 2) {
      uint32_t h[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) h[s] = (r + s < d) ? (uint32_t)col[r + s] : 0u;
      o.w[0] = h[0] | (h[1] << 16);
      o.w[1] = h[2] | (h[3] << 16);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) o.v[s] = (r + s < d) ? col[r + s] : (TX)0;
    }
  }
}

// Four consecutive elements X[r..r+3] of one column, all rows < d (no bounds
// logic, so a group of these loads issues back to back).  VEC: column base and
// r aligned for one vector load.
template <typename TX, bool VEC>
__device__ __forceinline__ void load4full(const TX* __restrict__ col, int64_t r, Raw4<TX>& o) {
  if constexpr (VEC) {
    if constexpr (sizeof(TX) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(col + r);
      const double2 b = *reinterpret_cast<const double2*>(col + r + 2);
      o.v[0] = a.x; o.v[1] = a.y; o.v[2] = b.x; o.v[3] = b.y;
    } else if constexpr (sizeof(TX) == 4) {
      const float4 a = *reinterpret_cast<const float4*>(col + r);
      o.v[0] = a.x; o.v[1] = a.y; o.v[2] = a.z; o.v[3] = a.w;
    } else {
      const uint2 a = *reinterpret_cast<const uint2*>(col + r);
      o.w[0] = a.x; o.w[1] = a.y;
    }
  } else if constexpr (sizeof(TX) == 2) {
    o.w[0] = (uint32_t)col[r] | ((uint32_t)col[r + 1] << 16);
    o.w[1] = (uint32_t)col[r + 2] | ((uint32_t)col[r + 3] << 16);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) o.v[s] = col[r + s];
  }
}

// Lane l's four B-operand values of one tile of the tile-major difference.
__device__ __forceinline__ void load_tile_b(const double* __restrict__ tile, int l, double* m) {
  const double2 a = *reinterpret_cast<const double2*>(tile + 2 * l);
  const double2 b = *reinterpret_cast<const double2*>(tile + 128 + 2 * l);
  m[0] = a.x; m[1] = a.y; m[2] = b.x; m[3] = b.y;
}

// The same rows where some may be >= d: addresses clamped to row d - 1, values
// of rows >= d set to 0 after the load.
template <typename TX>
__device__ __forceinline__ void load4tail(const TX* __restrict__ col, int64_t r, int64_t d,
                                          Raw4<TX>& o) {
  TX h[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const TX v = col[min(r + s, d - 1)];
    h[s] = r + s < d ? v : (TX)0;
  }
  if constexpr (sizeof(TX) == 2) {
    o.w[0] = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    o.w[1] = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) o.v[s] = h[s];
  }
}

// Offset of (row r, column j) in the tile-major inner-step difference with NS
// 16-column slices (layout described with tile_add in kernels.h).
__device__ __forceinline__ int64_t dl_off(int64_t r, int j, int NS) {
  const int rho = (int)(r & 15), q = rho >> 2, s = rho & 3;
  return ((r >> 4) * NS + (j >> 4)) * 256 + (s >> 1) * 128 + (q * 16 + (j & 15)) * 2 + (s & 1);
}

constexpr int KSTAGE = 8192;   // largest minibatch; its indices are staged in LDS

// Sum the NW waves' accumulators (NACC 16x16 tiles each) into red[0 .. NACC*256):
// every wave writes its own slot of slots[NW][NACC*256], one barrier, then the
// sum over waves in wave order (so the result does not depend on timing).
template <int NW, int NACC>
__device__ __forceinline__ void waves_to_lds(double* red, double* slots, const v4d* acc, int q,
                                             int li) {
  const int t = threadIdx.x, wave = t / 64;
  double* mine = slots + wave * (NACC * 256);
#pragma unroll
  for (int a = 0; a < NACC; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) mine[a * 256 + (4 * v + q) * 16 + li] = acc[a][v];
  __syncthreads();
  for (int e = t; e < NACC * 256; e += NW * 64) {
    double s = slots[e];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += slots[w * (NACC * 256) + e];
    red[e] = s;
  }
  __syncthreads();
}

// Same sum with a single NACC*256 buffer, accumulated one wave at a time in
// wave order (NW barriers; for kernels whose slots would not fit in LDS).
template <int NW, int NACC>
__device__ __forceinline__ void waves_to_lds_seq(double* red, const v4d* acc, int q, int li) {
  const int wave = threadIdx.x / 64;
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double& o = red[a * 256 + (4 * v + q) * 16 + li];
          o = (w == 0 ? 0.0 : o) + acc[a][v];
        }
    }
    __syncthreads();
  }
}

// out[c * PC + 16 (NTW y + u) + j] = scale_c * sum_r X[r, col(c)] M[r, 16 (NTW y + u) + j]
// for c < ncols, j < 16, u < NTW, y = blockIdx.y.  col(c) = idx[c] (GATHER)
// or c.  M is tile-major with NSM = ceil(p / 16) slices (the layout of the
// inner-step difference, zero-padded to pad16(d) x 16 NSM): each 16-row block
// of a 16-column slice is two contiguous 1 KB loads.  Output slices that the
// grid covers past NSM are written as zeros.  A workgroup owns MT tiles of 16
// columns of X and NTW 16-column slices of M (each M fetch feeds MT tiles);
// its NW waves split the rows.
// Each wave keeps two register stages of G 16-row blocks: the loads of the
// next stage are issued before the matrix-core work of the current one.
// Every load of the main loop reads an in-bounds address (invalid columns
// read column idx[0] or 0, whose output rows are not stored; a stage's
// blocks past the wave's range read its last block and skip their
// matrix-core work on a wave-uniform branch), so no load waits on a branch.
// The partial last block of rows (d % 16 != 0) is done on its own with
// clamped, masked X loads (M's padding rows are zero).  VEC: X columns
// aligned for vector loads.  R4 > 0 (with nt0 = 0): after the NTW full
// slices, 4 R4 more columns of M (from slice NTW) are done with 4x4x4 matrix
// cores instead of a whole padded 16-column slice; output columns from
// 16 NTW + 4 R4 up to PC are written as zeros.
template <typename TX, int NW, int NTW, int G, bool GATHER, bool VEC, int MT = 1, int R4 = 0>
__global__ __launch_bounds__(NW * 64) void k_xtm(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                 int64_t ncols, const int32_t* __restrict__ idx,
                                                 const double* __restrict__ M, int NSM,
                                                 const double* __restrict__ scale,
                                                 double* __restrict__ out, int PC) {
  constexpr int R4A = R4 > 0 ? R4 : 1;
  __shared__ double red[MT * NTW * 256];
  __shared__ double slots[MT == 1 ? NW * NTW * 256 : 1];
  __shared__ double red4[R4 > 0 ? MT * R4 * 64 : 1];
  const int t = threadIdx.x, wave = t / 64, l = t % 64;
  const int li = l % 16, q = l / 16;
  const int64_t tile = blockIdx.x;
  const int nt0 = blockIdx.y * NTW;
  const int NS = NSM;
  bool cval[MT];
  const TX* xcol[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int64_t c = (tile * MT + mt) * 16 + li;
    cval[mt] = c < ncols;
    const int64_t cc = cval[mt] ? c : 0;
    xcol[mt] = X + (GATHER ? (int64_t)idx[cc] : cc) * ld;
  }
  // this workgroup's slices; a slice past the last (NTW not dividing the slice
  // count) reads the last one and its output is not stored
  int sl[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) sl[u] = min(nt0 + u, NS - 1);
  v4d acc[MT * NTW];
#pragma unroll
  for (int a = 0; a < MT * NTW; ++a) acc[a] = v4d{0.0, 0.0, 0.0, 0.0};
  double acc4[MT * R4A];
#pragma unroll
  for (int a = 0; a < MT * R4A; ++a) acc4[a] = 0.0;
  const int l4 = 16 * q + (l & 3);   // lane of the tile that holds this lane's 4x4x4 B values
  const int64_t nblk = (d + 15) / 16, nfull = d / 16;
  const int64_t bpw = (nblk + NW - 1) / NW;
  const int64_t b0 = wave * bpw, b1 = min(nblk, b0 + bpw);
  const int64_t bend = min(b1, nfull);
  struct Stage {
    Raw4<TX> x[G][MT];
    double m[G][NTW][4];
    double m4[G][R4A][4];
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t blk = min(g + i, bend - 1);
      const int64_t r = blk * 16 + 4 * q;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) load4full<TX, VEC>(xcol[mt], r, S.x[i][mt]);
#pragma unroll
      for (int u = 0; u < NTW; ++u) load_tile_b(M + (blk * NS + sl[u]) * 256, l, S.m[i][u]);
#pragma unroll
      for (int g = 0; g < R4; ++g) load_tile_b(M + (blk * NS + NTW) * 256, l4 + 4 * g, S.m4[i][g]);
    }
  };
  auto compute = [&](const Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (g + i >= bend) break;
#pragma unroll
      for (int u = 0; u < NTW; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[mt * NTW + u] = mfma_f64(S.x[i][mt].get(s), S.m[i][u][s], acc[mt * NTW + u]);
#pragma unroll
      for (int g = 0; g < R4; ++g)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc4[mt * R4A + g] = mfma_f64_4(S.x[i][mt].get(s), S.m4[i][g][s], acc4[mt * R4A + g]);
    }
  };
  if (b0 < bend) {
    Stage A, B;
    load(A, b0);
    for (int64_t g = b0; g < bend; g += 2 * G) {
      load(B, g + G);
      __builtin_amdgcn_sched_barrier(0);
      compute(A, g);
      load(A, g + 2 * G);
      __builtin_amdgcn_sched_barrier(0);
      compute(B, g + G);
    }
  }
  if (nfull < nblk && b0 <= nfull && nfull < b1) {   // this wave owns the partial last block
    const int64_t r = nfull * 16 + 4 * q;
    Raw4<TX> x[MT];
    double m[NTW][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) load4tail<TX>(xcol[mt], r, d, x[mt]);
#pragma unroll
    for (int u = 0; u < NTW; ++u) load_tile_b(M + (nfull * NS + sl[u]) * 256, l, m[u]);
    double m4[R4A][4];
#pragma unroll
    for (int g = 0; g < R4; ++g) load_tile_b(M + (nfull * NS + NTW) * 256, l4 + 4 * g, m4[g]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int u = 0; u < NTW; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[mt * NTW + u] = mfma_f64(x[mt].get(s), m[u][s], acc[mt * NTW + u]);
#pragma unroll
      for (int g = 0; g < R4; ++g)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc4[mt * R4A + g] = mfma_f64_4(x[mt].get(s), m4[g][s], acc4[mt * R4A + g]);
    }
  }
  if constexpr (MT == 1)
    waves_to_lds<NW, NTW>(red, slots, acc, q, li);
  else
    waves_to_lds_seq<NW, MT * NTW>(red, acc, q, li);
  if constexpr (R4 > 0) {   // the 4x4x4 results, summed one wave at a time in wave order
    for (int w = 0; w < NW; ++w) {
      if (wave == w) {
#pragma unroll
        for (int a = 0; a < MT * R4; ++a)
          red4[a * 64 + l] = (w == 0 ? 0.0 : red4[a * 64 + l]) + acc4[a];
      }
      __syncthreads();
    }
    // lane ll holds row 4 ((ll % 16) / 4) + ll / 16 of the tile, column 4 g + ll % 4
    for (int e = t; e < MT * R4 * 64; e += NW * 64) {
      const int a = e / 64, mt = a / R4, g = a % R4, ll = e % 64;
      const int64_t cc = (tile * MT + mt) * 16 + 4 * ((ll % 16) / 4) + ll / 16;
      const int j = NTW * 16 + 4 * g + (ll & 3);
      if (cc < ncols && j < PC) out[cc * PC + j] = red4[e];
    }
    const int jz = NTW * 16 + 4 * R4, nz = PC - jz;   // padding columns
    for (int e = t; e < MT * 16 * nz; e += NW * 64) {
      const int64_t cc = tile * MT * 16 + e / nz;
      if (cc < ncols) out[cc * PC + jz + e % nz] = 0.0;
    }
  }
  // gathered: rows from ncols up to the next multiple of 16 are written as
  // zeros (the inner-step update reads whole 16-sample blocks)
  const int64_t nrows = GATHER ? (ncols + 15) / 16 * 16 : ncols;
  for (int e = t; e < MT * NTW * 256; e += NW * 64) {
    const int a = e / 256, mt = a / NTW, u = a % NTW, i = (e / 16) % 16, jj = e % 16;
    const int64_t cc = (tile * MT + mt) * 16 + i;
    if (cc < nrows && (nt0 + u) * 16 < PC) {
      const double sc = cc < ncols ? (scale ? scale[cc] : 1.0) : 0.0;
      out[cc * PC + (nt0 + u) * 16 + jj] = cc < ncols && nt0 + u < NSM ? sc * red[e] : 0.0;
    }
  }
}

// Four rows r..r+3 of one column with the row index clamped to d - 1 (for the
// last, ragged 64-row tile: rows >= d read row d - 1; their results are not
// stored).
template <typename TX>
__device__ __forceinline__ void load4clamp(const TX* __restrict__ col, int64_t r, int64_t d,
                                           Raw4<TX>& o) {
  if constexpr (sizeof(TX) == 2) {
    o.w[0] = (uint32_t)col[min(r, d - 1)] | ((uint32_t)col[min(r + 1, d - 1)] << 16);
    o.w[1] = (uint32_t)col[min(r + 2, d - 1)] | ((uint32_t)col[min(r + 3, d - 1)] << 16);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) o.v[s] = col[min(r + s, d - 1)];
  }
}

// Pass, second half: part[split][j * d + r] = sum_{c in split} X[r, c] T[c * PC + j].
// A workgroup owns 64 rows as four 16-row tiles whose rows interleave
// (tile mt holds rows r0 + 4 i + mt), so each lane fetches four consecutive
// rows of one column with a single vector load; all 16 NT columns; the 8 waves
// split the column range.  Splits hold kper columns, a multiple of 16, so only
// the last block of the last split can be partial; it is done on its own with
// clamped, masked loads.  The main loop keeps two register stages of G column
// blocks with every load in bounds (a stage's blocks past the wave's range
// read its last block and skip their matrix-core work on a wave-uniform
// branch).  The grid is remapped so that the row tiles of one split run on one
// XCD (workgroups go to the 8 XCDs in turn) and share its T rows in one L2.
// R4 > 0: after the NT full slices, 4 R4 more columns of T are done with
// 4x4x4 matrix cores instead of a whole padded 16-column slice.
template <typename TX, int NT, int G, bool VEC, int R4 = 0>
__global__ __launch_bounds__(512) void k_xt_part(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                 int64_t n, const double* __restrict__ T, int PC,
                                                 int p, double* __restrict__ part, int64_t kper) {
  constexpr int NW = 8, MTL = 4, R4A = R4 > 0 ? R4 : 1;
  __shared__ double red[MTL * NT * 256];
  __shared__ double red4[R4 > 0 ? MTL * R4 * 64 : 1];
  const int t = threadIdx.x, wave = t / 64, l = t % 64;
  const int lm = l % 16, q = l / 16;
  const int RT = gridDim.x, NSP = gridDim.y;
  int rt = blockIdx.x, split = blockIdx.y;
  if (RT % 8 == 0 && NSP % 8 == 0) {
    const int64_t w = blockIdx.x + (int64_t)RT * blockIdx.y;
    const int64_t k = w / 8;
    split = (int)((k / RT) * 8 + w % 8);
    rt = (int)(k % RT);
  }
  const int64_t r0 = (int64_t)rt * 64;
  const int64_t rbase = r0 + 4 * lm;
  const int64_t ks = split * kper;
  const int64_t ke = min(n, ks + kper);
  v4d acc[MTL * NT];
#pragma unroll
  for (int a = 0; a < MTL * NT; ++a) acc[a] = v4d{0.0, 0.0, 0.0, 0.0};
  double acc4[MTL * R4A];
#pragma unroll
  for (int a = 0; a < MTL * R4A; ++a) acc4[a] = 0.0;
  const int64_t nblk = ke > ks ? (ke - ks + 15) / 16 : 0;
  const int64_t nfull = ke > ks ? (ke - ks) / 16 : 0;
  const int64_t bpw = (nblk + NW - 1) / NW;
  const int64_t b0 = wave * bpw, b1 = min(nblk, b0 + bpw);
  const int64_t bend = min(b1, nfull);
  const double* __restrict__ tq = T + (ks + 4 * q) * PC + lm;
  // this lane's column of T for the 4x4x4 groups (lane 16 k + 4 blk + n holds column n)
  const double* __restrict__ tq4 = T + (ks + 4 * q) * PC + NT * 16 + (l & 3);
  const TX* __restrict__ xq = X + (ks + 4 * q) * ld;
  struct Stage {
    Raw4<TX> x[G][4];
    double nv[G][4][NT];
    double nv4[G][4][R4A];
  };
  auto compute = [&](const Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (g + i >= bend) break;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int mt = 0; mt < MTL; ++mt) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[mt * NT + nt] = mfma_f64(S.x[i][s].get(mt), S.nv[i][s][nt], acc[mt * NT + nt]);
#pragma unroll
          for (int g = 0; g < R4; ++g)
            acc4[mt * R4A + g] = mfma_f64_4(S.x[i][s].get(mt), S.nv4[i][s][g], acc4[mt * R4A + g]);
        }
    }
  };
  // the ragged last row tile loads row by row with clamped rows; the others
  // take one vector load per column
  auto run = [&](auto ragged) {
    constexpr bool RG = decltype(ragged)::value;
    auto load = [&](Stage& S, int64_t g) {
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int64_t blk = min(g + i, bend - 1);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const TX* __restrict__ col = xq + (blk * 16 + s) * ld;
          if constexpr (RG)
            load4clamp<TX>(col, rbase, d, S.x[i][s]);
          else
            load4full<TX, VEC>(col, rbase, S.x[i][s]);
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) S.nv[i][s][nt] = tq[(blk * 16 + s) * PC + nt * 16];
#pragma unroll
          for (int g = 0; g < R4; ++g) S.nv4[i][s][g] = tq4[(blk * 16 + s) * PC + 4 * g];
        }
      }
    };
    if (b0 < bend) {
      Stage A, B;
      load(A, b0);
      for (int64_t g = b0; g < bend; g += 2 * G) {
        load(B, g + G);
        __builtin_amdgcn_sched_barrier(0);
        compute(A, g);
        load(A, g + 2 * G);
        __builtin_amdgcn_sched_barrier(0);
        compute(B, g + G);
      }
    }
  };
  if (r0 + 64 > d)
    run(std::true_type{});
  else
    run(std::false_type{});
  if (nfull < nblk && b0 <= nfull && nfull < b1) {   // the partial last block of columns
    Raw4<TX> x[4];
    double nv[4][NT], nv4[4][R4A];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t kc = ks + nfull * 16 + 4 * q + s;
      const bool kv = kc < ke;
      const int64_t kcc = kv ? kc : ke - 1;
      load4clamp<TX>(X + kcc * ld, rbase, d, x[s]);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const double v = T[kcc * PC + nt * 16 + lm];
        nv[s][nt] = kv ? v : 0.0;
      }
#pragma unroll
      for (int g = 0; g < R4; ++g) {
        const double v = T[kcc * PC + NT * 16 + 4 * g + (l & 3)];
        nv4[s][g] = kv ? v : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mt = 0; mt < MTL; ++mt) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt * NT + nt] = mfma_f64(x[s].get(mt), nv[s][nt], acc[mt * NT + nt]);
#pragma unroll
        for (int g = 0; g < R4; ++g)
          acc4[mt * R4A + g] = mfma_f64_4(x[s].get(mt), nv4[s][g], acc4[mt * R4A + g]);
      }
  }
  waves_to_lds_seq<NW, MTL * NT>(red, acc, q, lm);
  for (int e = t; e < MTL * NT * 256; e += NW * 64) {
    const int mt = e / (NT * 256), nt = (e / 256) % NT, i = (e / 16) % 16, jj = e % 16;
    const int64_t r = r0 + 4 * i + mt;
    const int j = nt * 16 + jj;
    if (r < d && j < p) part[(int64_t)split * p * d + (int64_t)j * d + r] = red[e];
  }
  if constexpr (R4 > 0) {   // the 4x4x4 results, summed one wave at a time in wave order
    for (int w = 0; w < NW; ++w) {
      if (wave == w) {
#pragma unroll
        for (int a = 0; a < MTL * R4; ++a)
          red4[a * 64 + l] = (w == 0 ? 0.0 : red4[a * 64 + l]) + acc4[a];
      }
      __syncthreads();
    }
    // lane ll holds row 4 ((ll % 16) / 4) + ll / 16 of tile mt, column 4 g + ll % 4
    for (int e = t; e < MTL * R4 * 64; e += NW * 64) {
      const int a = e / 64, mt = a / R4, g = a % R4, ll = e % 64;
      const int64_t r = r0 + 4 * (4 * ((ll % 16) / 4) + ll / 16) + mt;
      const int j = NT * 16 + 4 * g + (ll & 3);
      if (r < d && j < p) part[(int64_t)split * p * d + (int64_t)j * d + r] = red4[e];
    }
  }
}

// out = alpha * sum_split part + beta * A + gamma * B (fixed summation order).
__global__ __launch_bounds__(NT) void k_reduce_y(const double* __restrict__ part, int nsplit,
                                                 int64_t cnt, double alpha,
                                                 const double* __restrict__ A, double beta,
                                                 const double* __restrict__ B, double gamma,
                                                 double* __restrict__ out) {
  // RG threads per element, each summing a consecutive quarter of the splits in
  // split order; the quarters are then added in order (a fixed order)
  constexpr int RG = 4, EPB = NT / RG;
  __shared__ double qs[RG][EPB];
  const int t = threadIdx.x, el = t % EPB, g = t / EPB;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const int per = (nsplit + RG - 1) / RG;
  const int k0 = min(nsplit, g * per), k1 = min(nsplit, k0 + per);
  double s = 0.0;
  if (e < cnt) {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) s += part[(int64_t)k * cnt + e];
  }
  qs[g][el] = s;
  __syncthreads();
  if (g == 0 && e < cnt) {
    double v = qs[0][el];
#pragma unroll
    for (int h = 1; h < RG; ++h) v += qs[h][el];
    v = alpha * v;
    if (A) v += beta * A[e];
    if (B) v += gamma * B[e];
    out[e] = v;
  }
}

// Four entries of one column from row r as FP32 (exact for FP32 and BF16 X):
// VEC reads rows r .. r + 3 (all < d) with one load, the scalar form reads rows
// past d as zero (addresses clamped to row d - 1).
template <typename TX, bool VEC>
__device__ __forceinline__ float4 col4(const TX* __restrict__ col, int64_t r, int64_t d) {
  static_assert(sizeof(TX) < 8, "FP32 or BF16 storage");
  if constexpr (VEC && sizeof(TX) == 4) {
    return *reinterpret_cast<const float4*>(col + r);
  } else if constexpr (VEC) {
    const uint2 a = *reinterpret_cast<const uint2*>(col + r);
    return make_float4(__uint_as_float(a.x << 16), __uint_as_float(a.x & 0xFFFF0000u),
                       __uint_as_float(a.y << 16), __uint_as_float(a.y & 0xFFFF0000u));
  } else {
    float v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float x = (float)ldx(col, min(r + s, d - 1));
      v[s] = r + s < d ? x : 0.f;
    }
    return make_float4(v[0], v[1], v[2], v[3]);
  }
}

__device__ __forceinline__ float f4at(const float4& v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// Orders a wave's LDS accesses around it (a wave's own LDS operations complete
// in issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inner-step update for a tile of 16 rows and the 16-column slice nt = blockIdx.y:
// Dl <- Dl - eta (G + lam Dl - U),  U[r, j] = sum_s X[r, idx[s]] C[s * PC + j].
// The NW waves split the b samples (indices staged in LDS) and load G sample
// blocks ahead.  For FP32 and BF16 X a block of 16 samples comes in with one
// load per lane (lane l: rows 4 (l % 4) .. + 3 of the tile from sample l / 4;
// VEC moves a piece past d back to rows d - 4 .. d - 1, the scalar form reads
// rows past d as zero) and the wave turns it around through its own LDS tile
// (two, alternating; pitch 20 floats, so the 64 lanes' writes meet 64 banks)
// into the matrix-core operand order; FP64 X is gathered entry by entry.
template <typename TX, int NW, int G, int PC, int NTW, int KS, bool DEFL = false,
          bool VEC = false>
__global__ __launch_bounds__(NW * 64) void k_step_update(const TX* __restrict__ X, int64_t ld,
                                                         int64_t d, int64_t b,
                                                         const int32_t* __restrict__ idx,
                                                         const double* __restrict__ C, int p,
                                                         const double* __restrict__ Gr,
                                                         double* __restrict__ Dl, double lam,
                                                         double eta, Deflation df) {
  __shared__ double red[NTW * 256];
  __shared__ double slots[NW * NTW * 256];
  __shared__ int sidx[KS];
  __shared__ double vs[DEFL ? 64 * 16 * NTW : 1];
  constexpr bool TURN = sizeof(TX) < 8;
  constexpr int XTP = 20;
  __shared__ __align__(16) float xtr[TURN ? NW : 1][2][TURN ? 16 * XTP : 4];
  const int t = threadIdx.x, wave = t / 64, l = t % 64;
  const int lm = l % 16, q = l / 16;
  // Workgroups go to the 8 XCDs in turn; the grid (a multiple of 8 tiles) is
  // remapped so each XCD owns a contiguous run of row tiles, and the two
  // 64-byte halves of a 128-byte line of a gathered column meet in one L2.
  const int64_t tile = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int64_t r0 = tile * 16;
  if (r0 >= d) return;
  const int nt0 = blockIdx.y * NTW;
  // the epilogue's operands are fetched now, so their latency overlaps the loop
  double e_dl[NTW], e_g[NTW];
  int64_t eo[NTW];
  bool eval[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int e = t + u * NW * 64;
    const int64_t er = r0 + (e % 256) / 16;
    const int ej = (nt0 + e / 256) * 16 + e % 16;
    eval[u] = e < NTW * 256 && er < d && ej < p;
    eo[u] = eval[u] ? dl_off(er, ej, PC / 16) : 0;
    e_dl[u] = eval[u] ? Dl[eo[u]] : 0.0;
    e_g[u] = eval[u] ? Gr[(int64_t)ej * d + er] : 0.0;
  }
  // the index list is padded to whole 16-sample blocks with a valid column
  const int64_t bpad = (b + 15) / 16 * 16;
  for (int64_t e = t; e < bpad; e += NW * 64) sidx[e] = idx[e < b ? e : 0];
  __syncthreads();
  // rows >= d read row d - 1 (their results are not stored)
  const TX* __restrict__ xrow = X + min(r0 + lm, d - 1);
  v4d acc[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t nblk = (b + 15) / 16;
  const int64_t bpw = (nblk + NW - 1) / NW;
  const int64_t b0 = wave * bpw, b1 = min(nblk, b0 + bpw);
  // Two register stages of G sample blocks each: the loads of the next stage
  // are issued before the matrix-core work of the current one, so a wave
  // always has a stage in flight.  C holds zero rows from b up to the next
  // multiple of 16 and the index list is padded with a valid column, so
  // samples past b need no mask; a stage's blocks past the wave's range read
  // the wave's last block (in bounds) and skip their matrix-core work on a
  // wave-uniform branch.
  const int* __restrict__ sq = sidx + 4 * q;
  const double* __restrict__ cq = C + (int64_t)(4 * q) * PC + nt0 * 16 + lm;
  const int lj = l >> 2, lr = 4 * (l & 3);   // this lane's sample and first row in a block
  const int64_t rr = r0 + lr;
  const int64_t rl = VEC && rr + 4 > d ? d - 4 : rr;
  struct Stage {
    float4 xv[TURN ? G : 1];
    TX x[TURN ? 1 : G][4];
    double nv[G][4][NTW];
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t blk = min(g + i, b1 - 1);
      const int* __restrict__ si = sq + blk * 16;
      const double* __restrict__ ci = cq + blk * 16 * PC;
      if constexpr (TURN) S.xv[i] = col4<TX, VEC>(X + (int64_t)sidx[blk * 16 + lj] * ld, rl, d);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if constexpr (!TURN) S.x[i][s] = xrow[(int64_t)si[s] * ld];
#pragma unroll
        for (int u = 0; u < NTW; ++u) S.nv[i][s][u] = ci[s * PC + u * 16];
      }
    }
  };
  auto compute = [&](const Stage& S, int64_t g, bool checked) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (checked && g + i >= b1) break;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (TURN) {
        float* __restrict__ wt = xtr[wave][(g + i) & 1];
        wt[(lr + 0) * XTP + lj] = S.xv[i].x;
        wt[(lr + 1) * XTP + lj] = S.xv[i].y;
        wt[(lr + 2) * XTP + lj] = S.xv[i].z;
        wt[(lr + 3) * XTP + lj] = S.xv[i].w;
        wave_sync();
        a = *reinterpret_cast<const float4*>(wt + lm * XTP + 4 * q);
        wave_sync();
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double xa;
        if constexpr (TURN)
          xa = (double)f4at(a, s);
        else
          xa = ldx(&S.x[i][s], 0);
#pragma unroll
        for (int u = 0; u < NTW; ++u) acc[u] = mfma_f64(xa, S.nv[i][s][u], acc[u]);
      }
    }
  };
  if (b0 < b1) {
    // whole pairs of stages first, with no branch between a stage's loads and
    // the work before its use (a guarded use lets the compiler move the loads
    // down to it, and the next stage's loads no longer overlap)
    Stage A, B;
    load(A, b0);
    int64_t g = b0;
    for (; g + 2 * G <= b1; g += 2 * G) {
      load(B, g + G);
      __builtin_amdgcn_sched_barrier(0);
      compute(A, g, false);
      load(A, g + 2 * G);
      __builtin_amdgcn_sched_barrier(0);
      compute(B, g + G, false);
    }
    if (g < b1) {
      compute(A, g, true);
      if (g + G < b1) {
        load(B, g + G);
        compute(B, g + G, true);
      }
    }
  }
  waves_to_lds<NW, NTW>(red, slots, acc, q, lm);
  if constexpr (DEFL) {
    // deflated columns: X_B C loses its part along Ud, Ud (Z_B C), with the
    // chunk partials of Z_B C (Z = Ud^T X) summed in chunk order
    for (int e = t; e < df.ns * 16 * NTW; e += NW * 64) {
      const int tq = e / (16 * NTW), j = nt0 * 16 + e % (16 * NTW);
      double v = 0.0;
      if (j < PC)
        for (int ks = 0; ks < df.nks; ++ks) v += df.Vp[((int64_t)ks * df.PCZ + tq) * PC + j];
      vs[e] = v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int e = t + u * NW * 64;
    if (!eval[u]) continue;
    double U = red[e];
    if constexpr (DEFL) {
      const int64_t er = r0 + (e % 256) / 16;
      const int jl = (e / 256) * 16 + e % 16;
      double c = 0.0;
      for (int tq = 0; tq < df.ns; ++tq) c += df.Ud[(int64_t)tq * d + er] * vs[tq * 16 * NTW + jl];
      U -= c;
    }
    Dl[eo[u]] = e_dl[u] - eta * (e_g[u] + lam * e_dl[u] - U);
  }
}

// Chunk partials of Z_B C for a deflated inner step: Vp[ks][t][j] =
// sum over samples s of chunk ks of Z[idx_s * PCZ + t] C[s * PC + j]
// (Z = X^T Ud, n x PCZ row-major); one 16 x 16 tile per workgroup.
constexpr int ZKS = 256;   // samples per chunk
__global__ __launch_bounds__(NT) void k_zbc(const double* __restrict__ Z, int PCZ,
                                            const int32_t* __restrict__ idx,
                                            const double* __restrict__ C, int PC, int64_t b,
                                            double* __restrict__ Vp) {
  const int t = blockIdx.x * 16 + threadIdx.x / 16, j = blockIdx.y * 16 + threadIdx.x % 16;
  const int64_t s0 = (int64_t)blockIdx.z * ZKS;
  const int64_t s1 = min(b, s0 + ZKS);
  double acc = 0.0;
  for (int64_t s = s0; s < s1; ++s) acc = fma(Z[(int64_t)idx[s] * PCZ + t], C[s * PC + j], acc);
  Vp[((int64_t)blockIdx.z * PCZ + t) * PC + j] = acc;
}

// The tile-major form (NS slices) of the d x p column-major W, zero-padded to
// pad16(d) x 16 NS; one thread per output element, in output order.
__global__ __launch_bounds__(NT) void k_cm_to_tile(const double* __restrict__ W, int64_t d,
                                                   int p, int NS, double* __restrict__ out,
                                                   int64_t cnt) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= cnt) return;
  const int64_t te = e / 256;
  const int w = (int)(e % 256), l = (w % 128) / 2, s = (w / 128) * 2 + w % 2;
  const int64_t r = (te / NS) * 16 + 4 * (l / 16) + s;
  const int j = (int)(te % NS) * 16 + l % 16;
  out[e] = r < d && j < p ? W[(int64_t)j * d + r] : 0.0;
}

// out[j d + r] = W[j d + r] + Dl(r, j), Dl tile-major.
__global__ __launch_bounds__(NT) void k_tile_add(int64_t d, int p, int NS,
                                                 const double* __restrict__ W,
                                                 const double* __restrict__ Dl,
                                                 double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= d * p) return;
  const int64_t r = e % d;
  const int j = (int)(e / d);
  out[e] = W[e] + Dl[dl_off(r, j, NS)];
}

// All draws of `steps` consecutive inner steps (from step t0) of one epoch:
// idx[(t - t0) * b + j], scale[...] for draw j of step t.
__global__ __launch_bounds__(NT) void k_draw(int64_t n, const uint64_t* __restrict__ cdf,
                                             uint32_t k0, uint32_t k1, uint32_t t0, int64_t steps,
                                             uint32_t epoch, uint32_t word3, int64_t b,
                                             int32_t* __restrict__ idx,
                                             double* __restrict__ scale) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= steps * b) return;
  const int64_t t = e / b, j = e % b;
  int64_t i;
  double sc;
  draw_one(cdf, n, k0, k1, (uint32_t)j, t0 + (uint32_t)t, epoch, word3, b, &i, &sc);
  idx[e] = (int32_t)i;
  scale[e] = sc;
}

__global__ __launch_bounds__(NT) void k_sample_only(int64_t n, const uint64_t* __restrict__ cdf,
                                                    uint32_t k0, uint32_t k1, uint32_t step,
                                                    uint32_t epoch, uint32_t word3, int64_t b,
                                                    int32_t* __restrict__ idx,
                                                    double* __restrict__ scale) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= b) return;
  int64_t i;
  double sc;
  draw_one(cdf, n, k0, k1, (uint32_t)j, step, epoch, word3, b, &i, &sc);
  idx[j] = (int32_t)i;
  scale[j] = sc;
}

// ---------------------------------------------------------------------------
// Tall-skinny Gram A^T B, stage 1: each workgroup sums a contiguous row range.
__global__ __launch_bounds__(NT) void k_gram_part(const double* __restrict__ A, int64_t rsa,
                                                  int64_t csa, int pa,
                                                  const double* __restrict__ B, int64_t rsb,
                                                  int64_t csb, int pb, int64_t rows, int64_t rpb,
                                                  double* __restrict__ part) {
  __shared__ double as[32][65];
  __shared__ double bs[32][65];
  const int t = threadIdx.x;
  const int cnt = pa * pb;
  const int64_t rb = (int64_t)blockIdx.x * rpb;
  const int64_t re = min(rows, rb + rpb);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t r0 = rb; r0 < re; r0 += 32) {
    for (int e = t; e < 32 * 64; e += NT) {
      const int rr = e % 32, c = e / 32;
      const int64_t r = r0 + rr;
      as[rr][c] = (r < re && c < pa) ? A[r * rsa + c * csa] : 0.0;
      bs[rr][c] = (r < re && c < pb) ? B[r * rsb + c * csb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int o = t + q * NT;
      if (o < cnt) {
        const int a = o % pa, bb = o / pa;
        double s = acc[q];
        for (int rr = 0; rr < 32; ++rr) s = fma(as[rr][a], bs[rr][bb], s);
        acc[q] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int o = t + q * NT;
    if (o < cnt) part[(int64_t)blockIdx.x * cnt + o] = acc[q];
  }
}

__global__ __launch_bounds__(NT) void k_part_reduce(const double* __restrict__ part, int nblk,
                                                    int cnt, double* __restrict__ out) {
  const int o = blockIdx.x * NT + threadIdx.x;
  if (o >= cnt) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * cnt + o];
  out[o] = s;
}

__global__ __launch_bounds__(NT) void k_sumsq_part(const double* __restrict__ A, int64_t count,
                                                   int64_t per, double* __restrict__ part) {
  __shared__ double ss[NT];
  const int t = threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = min(count, b0 + per);
  double s = 0.0;
  for (int64_t i = b0 + t; i < b1; i += NT) s = fma(A[i], A[i], s);
  ss[t] = s;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (t < k) ss[t] += ss[t + k];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = ss[0];
}

__global__ __launch_bounds__(NT) void k_sum_final(const double* __restrict__ part, int nb,
                                                  double* __restrict__ out) {
  __shared__ double ss[NT];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nb; b += NT) s += part[b];
  ss[t] = s;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (t < k) ss[t] += ss[t + k];
    __syncthreads();
  }
  if (t == 0) out[0] = ss[0];
}

// D = A M + beta C for a d x p block A (column-major, leading dimension d) and a
// p x q block M: one thread per row.  M sits in LDS with zero rows past p (and
// zero columns past q), so the row's entries of A can be fetched UNR at a time
// from clamped, in-bounds addresses and their latencies overlap; the extra
// products are exact zeros and the sums keep their order.
template <int PM>
__global__ __launch_bounds__(NT) void k_gemm_small(int64_t d, int p, int q,
                                                   const double* __restrict__ A,
                                                   const double* __restrict__ M, int ldm,
                                                   double* __restrict__ D, double beta,
                                                   const double* __restrict__ C) {
  constexpr int UNR = PM >= 48 ? 4 : 8;   // wide blocks: fewer loads ahead, no spills
  constexpr int LDM = 64 + UNR;           // LDS rows per column of M: p <= 64, rounded up to UNR
  __shared__ double ms[PM * LDM];
  const int t = threadIdx.x;
  for (int e = t; e < PM * LDM; e += NT) {
    const int i = e % LDM, j = e / LDM;
    ms[e] = (i < p && j < q) ? M[i + (int64_t)j * ldm] : 0.0;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * NT + t;
  if (row >= d) return;
  double acc[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) acc[j] = 0.0;
  for (int i0 = 0; i0 < p; i0 += UNR) {
    double a[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) a[u] = A[(int64_t)min(i0 + u, p - 1) * d + row];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int j = 0; j < PM; ++j) acc[j] = fma(a[u], ms[(i0 + u) + j * LDM], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < PM; ++j)
    if (j < q) {
      const int64_t e = (int64_t)j * d + row;
      D[e] = C ? acc[j] + beta * C[e] : acc[j];
    }
}

__global__ __launch_bounds__(NT) void k_lincomb(int64_t count, double a,
                                                const double* __restrict__ X, double b,
                                                const double* __restrict__ Y, double c,
                                                const double* __restrict__ Z,
                                                double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= count) return;
  double v = a * X[e];
  if (Y) v += b * Y[e];
  if (Z) v += c * Z[e];
  out[e] = v;
}

// ---------------------------------------------------------------------------
// Small dense kernels, one workgroup, m <= 64.
constexpr int SM = 64;
constexpr double CHOL_PIVOT_REL = 1e-14;

__global__ __launch_bounds__(NT) void k_chol_rinv(const double* __restrict__ G, int m,
                                                  double* __restrict__ Rinv,
                                                  int* __restrict__ info) {
  __shared__ double a[SM][SM];
  __shared__ double li[SM][SM];
  __shared__ double g0[SM];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < m * m; e += NT) {
    const int i = e % m, j = e / m;
    a[i][j] = 0.5 * (G[i + j * m] + G[j + i * m]);
    if (i == j) g0[i] = a[i][j];
  }
  __syncthreads();
  // a pivot at or below CHOL_PIVOT_REL of its diagonal entry: the block has
  // (numerically) lost rank, reported like a negative pivot
  for (int j = 0; j < m; ++j) {
    if (t == 0) {
      const double dj = a[j][j];
      if (!(dj > CHOL_PIVOT_REL * g0[j]) || !isfinite(dj)) {
        bad = 1;
        a[j][j] = 1.0;
      } else {
        a[j][j] = sqrt(dj);
      }
    }
    __syncthreads();
    const double piv = a[j][j];
    for (int i = j + 1 + t; i < m; i += NT) a[i][j] /= piv;
    __syncthreads();
    const int w = m - j - 1;
    for (int e = t; e < w * w; e += NT) {
      const int i = j + 1 + e % w, k = j + 1 + e / w;
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  // column c of L^{-1} by forward substitution; Rinv = (L^{-1})^T
  if (t < m) {
    const int c = t;
    for (int i = 0; i < c; ++i) li[i][c] = 0.0;
    li[c][c] = 1.0 / a[c][c];
    for (int i = c + 1; i < m; ++i) {
      double s = 0.0;
      for (int jj = c; jj < i; ++jj) s = fma(a[i][jj], li[jj][c], s);
      li[i][c] = -s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < m * m; e += NT) {
    const int i = e % m, j = e / m;  // Rinv[i][j] = Linv[j][i]
    Rinv[i + j * m] = li[j][i];
  }
  if (t == 0 && bad) *info = 1;  // sticky: cleared only by the host
}

// Cyclic Jacobi with round-robin ordering: in each round the disjoint pairs
// are rotated together (rows, then columns), which equals applying the
// rotations one after another.
__global__ __launch_bounds__(NT) void k_jacobi(const double* __restrict__ H, int m,
                                               double* __restrict__ vals,
                                               double* __restrict__ vecs) {
  // one double of padding per row: column walks (a[row][P] over rows) then hit
  // every LDS bank instead of one
  __shared__ double a[SM][SM + 1];
  __shared__ double v[SM][SM + 1];
  __shared__ double rc[SM / 2], rs[SM / 2];
  __shared__ int rp[SM / 2], rq[SM / 2];
  constexpr int NWJ = NT / 64;
  __shared__ double roff[NWJ], rtot[NWJ];
  __shared__ int stop;
  const int t = threadIdx.x;
  for (int e = t; e < m * m; e += NT) {
    const int i = e % m, j = e / m;
    a[i][j] = 0.5 * (H[i + j * m] + H[j + i * m]);
    v[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m2 = m + (m & 1);
  const int np = m2 / 2;
  const int nr = m2 - 1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    // stopping test: off-diagonal and total squared mass, summed within each wave
    // by shuffles and then over the NWJ waves in a fixed order
    double off = 0.0, tot = 0.0;
    for (int e = t; e < m * m; e += NT) {
      const int i = e % m, j = e / m;
      const double x = a[i][j] * a[i][j];
      tot += x;
      if (i != j) off += x;
    }
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) {
      off += __shfl_down(off, k, 64);
      tot += __shfl_down(tot, k, 64);
    }
    if (t % 64 == 0) {
      roff[t / 64] = off;
      rtot[t / 64] = tot;
    }
    __syncthreads();
    if (t == 0) {
      double so = roff[0], st = rtot[0];
#pragma unroll
      for (int w = 1; w < NWJ; ++w) {
        so += roff[w];
        st += rtot[w];
      }
      stop = (so <= 1e-32 * st) || m < 2;
    }
    __syncthreads();
    if (stop) break;
    for (int r = 0; r < nr; ++r) {
      if (t < np) {
        int P, Q;
        if (t == 0) {
          P = r;
          Q = m2 - 1;
        } else {
          P = (r + t) % nr;
          Q = (r - t + nr) % nr;
        }
        double c = 1.0, s = 0.0;
        if (P < m && Q < m) {
          const double apq = a[P][Q];
          if (fabs(apq) > 1e-300) {
            const double tau = (a[Q][Q] - a[P][P]) / (2.0 * apq);
            const double tt =
                tau == 0.0 ? 1.0 : copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        } else {
          P = Q = -1;
        }
        rp[t] = P;
        rq[t] = Q;
        rc[t] = c;
        rs[t] = s;
      }
      __syncthreads();
      for (int e = t; e < np * m; e += NT) {  // rows P, Q <- J^T A
        const int pi = e / m, col = e % m;
        const int P = rp[pi], Q = rq[pi];
        if (P >= 0) {
          const double c = rc[pi], s = rs[pi];
          const double aP = a[P][col], aQ = a[Q][col];
          a[P][col] = c * aP - s * aQ;
          a[Q][col] = s * aP + c * aQ;
        }
      }
      __syncthreads();
      for (int e = t; e < np * m; e += NT) {  // columns P, Q <- A J, V J
        const int pi = e / m, row = e % m;
        const int P = rp[pi], Q = rq[pi];
        if (P >= 0) {
          const double c = rc[pi], s = rs[pi];
          const double aP = a[row][P], aQ = a[row][Q];
          // the entry the rotation annihilates is stored as an exact zero
          const bool zP = row == Q && s != 0.0, zQ = row == P && s != 0.0;
          a[row][P] = zP ? 0.0 : c * aP - s * aQ;
          a[row][Q] = zQ ? 0.0 : s * aP + c * aQ;
          const double vP = v[row][P], vQ = v[row][Q];
          v[row][P] = c * vP - s * vQ;
          v[row][Q] = s * vP + c * vQ;
        }
      }
      __syncthreads();
    }
  }
  // descending order, ties by index; eigenvector sign: largest |entry| positive
  if (t < m) {
    const double di = a[t][t];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double dj = a[j][j];
      if (dj > di || (dj == di && j < t)) ++rank;
    }
    int am = 0;
    double best = -1.0;
    for (int row = 0; row < m; ++row) {
      const double x = fabs(v[row][t]);
      if (x > best) {
        best = x;
        am = row;
      }
    }
    const double sg = v[am][t] < 0.0 ? -1.0 : 1.0;
    vals[rank] = di;
    for (int row = 0; row < m; ++row) vecs[row + rank * m] = sg * v[row][t];
  }
}

__global__ __launch_bounds__(NT) void k_shift_inverse(const double* __restrict__ vals,
                                                      const double* __restrict__ Q, int m,
                                                      double lam, double* __restrict__ M) {
  const int t = threadIdx.x;
  for (int e = t; e < m * m; e += NT) {
    const int i = e % m, j = e / m;
    double s = 0.0;
    for (int l = 0; l < m; ++l) s += Q[i + l * m] * Q[j + l * m] / (lam - vals[l]);
    M[e] = s;
  }
}

__global__ __launch_bounds__(NT) void k_residual_norms(const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       const double* __restrict__ theta,
                                                       int64_t d, double* __restrict__ out) {
  __shared__ double ss[NT];
  const int i = blockIdx.x, t = threadIdx.x;
  const double th = theta[i];
  double s = 0.0;
  for (int64_t r = t; r < d; r += NT) {
    const double x = A[(int64_t)i * d + r] - th * B[(int64_t)i * d + r];
    s = fma(x, x, s);
  }
  ss[t] = s;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (t < k) ss[t] += ss[t + k];
    __syncthreads();
  }
  if (t == 0) out[i] = sqrt(ss[0]);
}

// The signed value of the winning entry travels with its magnitude and index
// through the reduction: the column is rewritten in place, so no thread may
// look the entry up in memory again (its owner may already have flipped it).
__global__ __launch_bounds__(NT) void k_sign_fix(double* __restrict__ U, int64_t d) {
  __shared__ double bv[NT], bs[NT];
  __shared__ int64_t bi[NT];
  const int t = threadIdx.x;
  double* col = U + (int64_t)blockIdx.x * d;
  double best = -1.0, sv = 0.0;
  int64_t am = 0;
  for (int64_t r = t; r < d; r += NT) {
    const double v = col[r];
    const double x = fabs(v);
    if (x > best) {
      best = x;
      sv = v;
      am = r;
    }
  }
  bv[t] = best;
  bs[t] = sv;
  bi[t] = am;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (t < k) {
      const double o = bv[t + k];
      const int64_t oi = bi[t + k];
      if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
        bv[t] = o;
        bs[t] = bs[t + k];
        bi[t] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = bs[0] < 0.0 ? -1.0 : 1.0;
  for (int64_t r = t; r < d; r += NT) col[r] *= sg;
}

__global__ __launch_bounds__(NT) void k_fill_u32(uint32_t* __restrict__ p, int64_t words,
                                                  uint32_t v) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < words;
       e += (int64_t)gridDim.x * NT)
    p[e] = v;
}

__global__ void k_fill_tail(unsigned char* __restrict__ p, int64_t bytes, unsigned char v) {
  if (threadIdx.x < bytes) p[threadIdx.x] = v;
}

inline unsigned nblocks(int64_t count, int per = NT) {
  return (unsigned)((count + per - 1) / per);
}

}  // namespace

// Launch a kernel; with probe events, time exactly this kernel's execution.
template <typename K, typename... A>
static void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, const Probe& pr, A... args) {
  if (pr.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pr.start, pr.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

#define LR_DISPATCH_DT(dt, TX, ...)   \
  switch (dt) {                       \
    case 0: {                         \
      using TX = double;              \
      __VA_ARGS__;                    \
    } break;                          \
    case 1: {                         \
      using TX = float;               \
      __VA_ARGS__;                    \
    } break;                          \
    case 2: {                         \
      using TX = uint16_t;            \
      __VA_ARGS__;                    \
    } break;                          \
    default:                          \
      return hipErrorInvalidValue;    \
  }

#define LR_DISPATCH_PM(p, PM, ...)                                  \
  if ((p) <= 8) {                                                   \
    constexpr int PM = 8;                                           \
    __VA_ARGS__;                                                    \
  } else if ((p) <= 16) {                                           \
    constexpr int PM = 16;                                          \
    __VA_ARGS__;                                                    \
  } else if ((p) <= 24) {                                           \
    constexpr int PM = 24;                                          \
    __VA_ARGS__;                                                    \
  } else if ((p) <= 32) {                                           \
    constexpr int PM = 32;                                          \
    __VA_ARGS__;                                                    \
  } else if ((p) <= 48) {                                           \
    constexpr int PM = 48;                                          \
    __VA_ARGS__;                                                    \
  } else if ((p) <= 64) {                                           \
    constexpr int PM = 64;                                          \
    __VA_ARGS__;                                                    \
  } else {                                                          \
    return hipErrorInvalidValue;                                    \
  }

hipError_t colnorms(const XView& X, double* w, int* bad, hipStream_t st) {
  LR_DISPATCH_DT(X.dt, TX,
                 k_colnorm<TX><<<nblocks(X.n, CN_COLS), NT, 0, st>>>((const TX*)X.v, X.ld, X.d,
                                                                     X.n, w, bad));
  return hipGetLastError();
}

hipError_t build_table(const double* w, int64_t n, uint64_t* cdf, double* fro2, double* scratch,
                       hipStream_t st) {
  const int64_t nb = (n + TB - 1) / TB;
  double* pmax = scratch;
  double* psum = scratch + nb;
  double* stats = scratch + 2 * nb;
  uint64_t* bsum = (uint64_t*)(scratch + 2 * nb + 2);
  k_wstats<<<(unsigned)nb, NT, 0, st>>>(w, n, pmax, psum);
  k_wfinal<<<1, NT, 0, st>>>(pmax, psum, nb, stats, fro2);
  k_quant<<<(unsigned)nb, NT, 0, st>>>(w, n, stats, cdf, bsum);
  k_scan_bsum<<<1, NT, 0, st>>>(bsum, nb);
  k_scan_local<<<(unsigned)nb, NT, 0, st>>>(cdf, n, bsum);
  return hipGetLastError();
}

hipError_t gaussian(double* S, int64_t d, int p, uint64_t seed, uint32_t word3, hipStream_t st) {
  k_gauss<<<nblocks(d * p), NT, 0, st>>>(S, d, p, (uint32_t)seed, (uint32_t)(seed >> 32), word3);
  return hipGetLastError();
}

#define LR_DISPATCH_NT(p, NTV, ...)   \
  if ((p) <= 16) {                    \
    constexpr int NTV = 1;            \
    __VA_ARGS__;                      \
  } else if ((p) <= 32) {             \
    constexpr int NTV = 2;            \
    __VA_ARGS__;                      \
  } else if ((p) <= 48) {             \
    constexpr int NTV = 3;            \
    __VA_ARGS__;                      \
  } else if ((p) <= 64) {             \
    constexpr int NTV = 4;            \
    __VA_ARGS__;                      \
  } else {                            \
    return hipErrorInvalidValue;      \
  }

int pad16(int p) { return ((p + 15) / 16) * 16; }

// Vector loads of four consecutive rows need the column start aligned.
static bool x_vec_ok(const XView& X) {
  const uintptr_t base = (uintptr_t)X.v;
  if (X.dt == 0) return X.ld % 2 == 0 && base % 16 == 0;
  if (X.dt == 1) return X.ld % 4 == 0 && base % 16 == 0;
  return X.ld % 4 == 0 && base % 8 == 0;
}

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Column splits of the pass's second half: about 512 workgroups of 64 rows
// (longer column runs per workgroup streamed 10% faster than about 2048 at
// 2048 x 200000 FP32, and leave a quarter of the partial sums to reduce).
int pass_nsplit(int64_t d, int64_t n) {
  const int64_t tiles = (d + 63) / 64;
  return (int)clampi((512 + tiles - 1) / tiles, 1, std::max<int64_t>(1, (n + 127) / 128));
}

template <int NW, int NTW, int G, bool GATHER, int MT = 1, int R4 = 0>
static hipError_t launch_xtm(const XView& X, int64_t ncols, const int32_t* idx, const double* M,
                             int p, const double* scale, double* out, int PC, hipStream_t st,
                             const Probe& pr) {
  if ((uintptr_t)M % 16) return hipErrorInvalidValue;   // tile loads are 16-byte vectors
  const bool vec = x_vec_ok(X);
  const int nt = (p + 15) / 16;   // slices of M's tile layout
  dim3 grid((unsigned)((ncols + 16 * MT - 1) / (16 * MT)),
            R4 > 0 ? 1u : (unsigned)((nt + NTW - 1) / NTW));
  LR_DISPATCH_DT(X.dt, TX, {
    if (vec)
      launch(k_xtm<TX, NW, NTW, G, GATHER, true, MT, R4>, grid, dim3(NW * 64), st, pr,
             (const TX*)X.v, X.ld, X.d, ncols, idx, M, nt, scale, out, PC);
    else
      launch(k_xtm<TX, NW, NTW, G, GATHER, false, MT, R4>, grid, dim3(NW * 64), st, pr,
             (const TX*)X.v, X.ld, X.d, ncols, idx, M, nt, scale, out, PC);
  });
  return hipGetLastError();
}

// The pass reads every column once; MT column tiles per workgroup share each
// fetch of W.  Two tiles (32 columns) keep four waves per SIMD resident, which
// beat four tiles by 9% at p = 20 on 2048 x 200000 FP32 X (490 against 538 us).
hipError_t pass_xtw(const XView& X, const double* W, int p, double* T, int PC, double* Wtile,
                    hipStream_t st, const Probe& pr) {
  if (p > 64 || pad16(p) > PC || !Wtile) return hipErrorInvalidValue;
  // W to the tile-major form (zero-padded), PC = pad16(p) slices of 16 columns
  const int PCw = pad16(p);
  const int64_t cnt = (X.d + 15) / 16 * 16 * PCw;
  k_cm_to_tile<<<nblocks(cnt), NT, 0, st>>>(W, X.d, p, PCw / 16, Wtile, cnt);
  // whole 16-column slices, and the last p % 16 <= 12 columns as 4x4x4 groups
  const int rem = p % 16, r4 = rem > 0 && rem <= 12 && p > 16 ? (rem + 3) / 4 : 0;
  const int full = r4 > 0 ? p / 16 : (p + 15) / 16;
#define LR_PASS1(NF, R)                                                                     \
  if (full == NF && r4 == R)                                                                \
    return launch_xtm<8, NF, (NF == 1 && R == 0 ? 2 : 1), false,                          \
                      (NF == 2 && R == 0 ? 4 : 2), R>(                                       \
        X, X.n, nullptr, Wtile, p, nullptr, T, PC, st, pr);
  LR_PASS1(1, 0) LR_PASS1(1, 1) LR_PASS1(1, 2) LR_PASS1(1, 3)
  LR_PASS1(2, 0) LR_PASS1(2, 1) LR_PASS1(2, 2) LR_PASS1(2, 3)
  LR_PASS1(3, 0) LR_PASS1(3, 1) LR_PASS1(3, 2) LR_PASS1(3, 3) LR_PASS1(4, 0)
#undef LR_PASS1
  return hipErrorInvalidValue;
}

hipError_t pass_xt(const XView& X, const double* T, int PC, int p, const PassBufs& pb,
                   double alpha, const double* A, double beta, const double* B, double gamma,
                   double* out, hipStream_t st, const Probe& pr) {
  if (p > 64 || pad16(p) > PC) return hipErrorInvalidValue;
  dim3 grid((unsigned)((X.d + 63) / 64), (unsigned)pb.nsplit);
  // columns per split: a multiple of 16, so only the last block can be partial
  const int64_t kper = ((X.n + pb.nsplit - 1) / pb.nsplit + 15) / 16 * 16;
  const bool vec = x_vec_ok(X);
  // whole 16-column slices, and the last p % 16 <= 12 columns as 4x4x4 groups
  const int rem = p % 16, r4 = rem > 0 && rem <= 12 && p > 16 ? (rem + 3) / 4 : 0;
  const int full = r4 > 0 ? p / 16 : (p + 15) / 16;
  bool done = false;
#define LR_PASS2(NF, R)                                                                      \
  if (!done && full == NF && r4 == R) {                                                      \
    done = true;                                                                             \
    LR_DISPATCH_DT(X.dt, TX, {                                                               \
      if (vec)                                                                               \
        launch(k_xt_part<TX, NF, 1, true, R>, grid, dim3(512), st, pr, (const TX*)X.v, X.ld, \
               X.d, X.n, T, PC, p, pb.Ypart, kper);                                          \
      else                                                                                   \
        launch(k_xt_part<TX, NF, 1, false, R>, grid, dim3(512), st, pr, (const TX*)X.v,      \
               X.ld, X.d, X.n, T, PC, p, pb.Ypart, kper);                                    \
    });                                                                                      \
  }
  LR_PASS2(1, 0) LR_PASS2(1, 1) LR_PASS2(1, 2) LR_PASS2(1, 3)
  LR_PASS2(2, 0) LR_PASS2(2, 1) LR_PASS2(2, 2) LR_PASS2(2, 3)
  LR_PASS2(3, 0) LR_PASS2(3, 1) LR_PASS2(3, 2) LR_PASS2(3, 3) LR_PASS2(4, 0)
#undef LR_PASS2
  if (!done) return hipErrorInvalidValue;
  const int64_t cnt = X.d * p;
  k_reduce_y<<<nblocks(cnt, NT / 4), NT, 0, st>>>(pb.Ypart, pb.nsplit, cnt, alpha, A, beta, B,
                                                  gamma, out);
  return hipGetLastError();
}

hipError_t draw_chunk(int64_t n, const uint64_t* cdf, uint64_t seed, uint32_t t0, int64_t steps,
                      uint32_t epoch, uint32_t word3, int64_t b, int32_t* idx, double* scale,
                      hipStream_t st) {
  k_draw<<<nblocks(steps * b), NT, 0, st>>>(n, cdf, (uint32_t)seed, (uint32_t)(seed >> 32), t0,
                                             steps, epoch, word3, b, idx, scale);
  return hipGetLastError();
}

// Workgroup size follows the problem: each wave gets about one prefetch group
// of 16-row blocks, so small problems launch small workgroups that share a CU
// with the kernels of other requests instead of holding it alone.
hipError_t step_dot(const XView& X, int p, int64_t b, const int32_t* idx, const double* scale,
                    const double* Dl, double* C, int PC, hipStream_t st, const Probe& pr) {
  if (p > 64 || pad16(p) > PC) return hipErrorInvalidValue;
  // four waves per workgroup: faster than eight by 5-8% at d = 512 ... 4096 (two
  // or sixteen waves, and other stage depths, are slower still)
  return launch_xtm<4, 1, 2, true>(X, b, idx, Dl, p, scale, C, PC, st, pr);
}

int zbc_chunks(int64_t b) { return (int)((b + ZKS - 1) / ZKS); }

hipError_t tile_add(int64_t d, int p, int PC, const double* W, const double* Dl, double* out,
                    hipStream_t st) {
  if (p > PC || PC % 16) return hipErrorInvalidValue;
  k_tile_add<<<nblocks(d * p), NT, 0, st>>>(d, p, PC / 16, W, Dl, out);
  return hipGetLastError();
}

hipError_t step_update(const XView& X, int p, int64_t b, const int32_t* idx, const double* C,
                       int PC, const double* G, double* Dl, double lam, double eta,
                       hipStream_t st, const Probe& pr, const Deflation& df) {
  if (p > 64 || b > KSTAGE || pad16(p) != PC) return hipErrorInvalidValue;
  const bool defl = df.ns > 0;
  if (defl) {
    if (df.ns > 64 || df.PCZ != pad16(df.ns) || !df.Z || !df.Vp || !df.Ud ||
        df.nks != zbc_chunks(b))
      return hipErrorInvalidValue;
    k_zbc<<<dim3((unsigned)(df.PCZ / 16), (unsigned)(PC / 16), (unsigned)df.nks), NT, 0, st>>>(
        df.Z, df.PCZ, idx, C, PC, b, df.Vp);
  }
  // one 16-column slice per workgroup: twice the gathers of one slice per
  // row tile, but twice the workgroups, which this latency-bound step needs
  dim3 grid((unsigned)(((X.d + 15) / 16 + 7) / 8 * 8), (unsigned)((p + 15) / 16));
  // waves split the samples: as many as give each about one prefetch group
  // FP32 / BF16 X in pieces of 4 rows: aligned columns, d a multiple of 4
  const bool vec = X.dt != 0 && X.ld % 4 == 0 && X.d % 4 == 0 &&
                   (uintptr_t)X.v % (X.dt == 1 ? 16 : 8) == 0;
#define LR_UPDATE_V(NWV, GV, KSV, DF, VC)                                                       \
  launch(k_step_update<TX, NWV, GV, 16 * NTV, 1, KSV, DF, VC>, grid, dim3(NWV * 64), st, pr,   \
         (const TX*)X.v, X.ld, X.d, b, idx, C, p, G, Dl, lam, eta, df)
#define LR_UPDATE(NWV, GV, KSV)                                                                \
  LR_DISPATCH_DT(X.dt, TX, LR_DISPATCH_NT(p, NTV, {                                            \
    if constexpr (sizeof(TX) < 8) {                                                            \
      if (defl && vec)                                                                         \
        LR_UPDATE_V(NWV, GV, KSV, true, true);                                                 \
      else if (defl)                                                                           \
        LR_UPDATE_V(NWV, GV, KSV, true, false);                                                \
      else if (vec)                                                                            \
        LR_UPDATE_V(NWV, GV, KSV, false, true);                                                \
      else                                                                                     \
        LR_UPDATE_V(NWV, GV, KSV, false, false);                                               \
    } else {                                                                                   \
      if (defl)                                                                                \
        LR_UPDATE_V(NWV, GV, KSV, true, false);                                                \
      else                                                                                     \
        LR_UPDATE_V(NWV, GV, KSV, false, false);                                               \
    }                                                                                          \
  }))
  // stage depth (blocks per stage) measured at d = 2048: 2 for small minibatches,
  // 1 for large ones (16 waves each with 2 stages in flight)
  if (b <= 256) {
    LR_UPDATE(4, 2, 256);
  } else if (b <= 512) {
    LR_UPDATE(8, 2, 512);
  } else {
    LR_UPDATE(16, 1, KSTAGE);
  }
#undef LR_UPDATE
#undef LR_UPDATE_V
  return hipGetLastError();
}

hipError_t sample_only(int64_t n, const uint64_t* cdf, uint64_t seed, uint32_t step,
                       uint32_t epoch, uint32_t word3, int64_t b, int32_t* idx, double* scale,
                       hipStream_t st) {
  k_sample_only<<<nblocks(b), NT, 0, st>>>(n, cdf, (uint32_t)seed, (uint32_t)(seed >> 32), step,
                                           epoch, word3, b, idx, scale);
  return hipGetLastError();
}

int gram_nblk(int64_t rows) {
  int64_t nb = (rows + 63) / 64;
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t gram(const double* A, int64_t rsa, int64_t csa, int pa, const double* B, int64_t rsb,
                int64_t csb, int pb, int64_t rows, double* part, double* G, hipStream_t st) {
  if (pa > 64 || pb > 64) return hipErrorInvalidValue;
  const int nb = gram_nblk(rows);
  const int64_t rpb = (rows + nb - 1) / nb;
  k_gram_part<<<nb, NT, 0, st>>>(A, rsa, csa, pa, B, rsb, csb, pb, rows, rpb, part);
  k_part_reduce<<<nblocks(pa * pb), NT, 0, st>>>(part, nb, pa * pb, G);
  return hipGetLastError();
}

hipError_t sumsq(const double* A, int64_t count, double* part, double* out, hipStream_t st) {
  int64_t nb = (count + 4095) / 4096;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  const int64_t per = (count + nb - 1) / nb;
  k_sumsq_part<<<(unsigned)nb, NT, 0, st>>>(A, count, per, part);
  k_sum_final<<<1, NT, 0, st>>>(part, (int)nb, out);
  return hipGetLastError();
}

hipError_t gemm_small(int64_t d, int p, int q, const double* A, const double* M, int ldm, double* D,
                      double beta, const double* C, hipStream_t st) {
  if (p > 64) return hipErrorInvalidValue;
  LR_DISPATCH_PM(q, PM,
                 k_gemm_small<PM><<<nblocks(d), NT, 0, st>>>(d, p, q, A, M, ldm, D, beta, C));
  return hipGetLastError();
}

hipError_t lincomb(int64_t count, double a, const double* X, double b, const double* Y, double c,
                   const double* Z, double* out, hipStream_t st) {
  k_lincomb<<<nblocks(count), NT, 0, st>>>(count, a, X, b, Y, c, Z, out);
  return hipGetLastError();
}

hipError_t chol_rinv(const double* G, int m, double* Rinv, int* info, hipStream_t st) {
  if (m > SM) return hipErrorInvalidValue;
  k_chol_rinv<<<1, NT, 0, st>>>(G, m, Rinv, info);
  return hipGetLastError();
}

hipError_t eigh(const double* H, int m, double* vals, double* vecs, hipStream_t st) {
  if (m > SM) return hipErrorInvalidValue;
  k_jacobi<<<1, NT, 0, st>>>(H, m, vals, vecs);
  return hipGetLastError();
}

hipError_t shift_inverse(const double* vals, const double* Q, int m, double lam, double* M,
                         hipStream_t st) {
  k_shift_inverse<<<1, NT, 0, st>>>(vals, Q, m, lam, M);
  return hipGetLastError();
}

hipError_t residual_norms(const double* A, const double* B, const double* theta, int64_t d, int m,
                          double* out, hipStream_t st) {
  k_residual_norms<<<m, NT, 0, st>>>(A, B, theta, d, out);
  return hipGetLastError();
}

hipError_t fill_bytes(void* p, size_t bytes, unsigned char byte, hipStream_t st) {
  if ((uintptr_t)p % 4) return hipErrorInvalidValue;
  const int64_t words = (int64_t)(bytes / 4);
  const uint32_t v = byte * 0x01010101u;
  if (words > 0)
    k_fill_u32<<<(unsigned)std::min<int64_t>(nblocks(words), 4096), NT, 0, st>>>(
        (uint32_t*)p, words, v);
  if (bytes % 4)
    k_fill_tail<<<1, 4, 0, st>>>((unsigned char*)p + words * 4, (int64_t)(bytes % 4), byte);
  return hipGetLastError();
}

hipError_t sign_fix(double* U, int64_t d, int k, hipStream_t st) {
  k_sign_fix<<<k, NT, 0, st>>>(U, d);
  return hipGetLastError();
}

}  // namespace lr
