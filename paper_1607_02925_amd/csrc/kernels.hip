// gfx950 kernels of the shift-and-invert low-rank path.  All arithmetic is
// FP64; X is read in its storage type (f64, f32 or bf16 bit patterns) and
// widened on load.  See kernels.h for the contract of each launcher.
#include "kernels.h"

#include <math.h>

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
template <typename TX>
__global__ __launch_bounds__(NT) void k_colnorm(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                int64_t n, double* __restrict__ w,
                                                int* __restrict__ bad) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const TX* col = X + i * ld;
  double s = 0.0;
  for (int64_t r = 0; r < d; ++r) {
    const double x = ldx(col, r);
    const double sq = x * x;
    s = s + sq;
  }
  w[i] = s;
  if (!isfinite(s)) atomicOr(bad, 1);
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
// Pass, first half: T = X^T W.  One thread per column of X; a workgroup
// stages a 16-row x 256-column slab of X in LDS with coalesced loads, and
// every thread reads the wave-uniform W values as scalars.
constexpr int XTW_RC = 16;
template <typename TX, int PM>
__global__ __launch_bounds__(NT) void k_xtw(const TX* __restrict__ X, int64_t ld, int64_t d,
                                            int64_t n, int p, const double* __restrict__ W,
                                            double* __restrict__ T) {
  __shared__ double xs[XTW_RC][NT + 1];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * NT;
  double acc[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) acc[j] = 0.0;
  for (int64_t r0 = 0; r0 < d; r0 += XTW_RC) {
#pragma unroll
    for (int e0 = 0; e0 < NT * XTW_RC; e0 += NT) {
      const int e = e0 + t;
      const int cc = e / XTW_RC, rr = e % XTW_RC;
      const int64_t cg = c0 + cc, r = r0 + rr;
      xs[rr][cc] = (cg < n && r < d) ? ldx(X, cg * ld + r) : 0.0;
    }
    __syncthreads();
    const int rmax = (int)min<int64_t>(XTW_RC, d - r0);
    for (int rr = 0; rr < rmax; ++rr) {
      const double xv = xs[rr][t];
      const double* wr = W + r0 + rr;
#pragma unroll
      for (int j = 0; j < PM; ++j)
        if (j < p) acc[j] = fma(xv, wr[(int64_t)j * d], acc[j]);
    }
    __syncthreads();
  }
  const int64_t col = c0 + t;
  if (col < n) {
#pragma unroll
    for (int j = 0; j < PM; ++j)
      if (j < p) T[col * p + j] = acc[j];
  }
}

// Pass, second half: Ypart[split] = X[:, split cols] T[split cols, :].
// One thread per row; X loads are coalesced along rows, T rows are uniform.
template <typename TX, int PM>
__global__ __launch_bounds__(NT) void k_xt(const TX* __restrict__ X, int64_t ld, int64_t d,
                                           int64_t n, int p, const double* __restrict__ T,
                                           int64_t cps, double* __restrict__ Ypart) {
  const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int split = blockIdx.y;
  const int64_t c0 = (int64_t)split * cps;
  const int64_t c1 = min(n, c0 + cps);
  double acc[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) acc[j] = 0.0;
  const int64_t rr = row < d ? row : d - 1;
  for (int64_t i = c0; i < c1; ++i) {
    const double xv = ldx(X, i * ld + rr);
    const double* ti = T + i * p;
#pragma unroll
    for (int j = 0; j < PM; ++j)
      if (j < p) acc[j] = fma(xv, ti[j], acc[j]);
  }
  if (row < d) {
    double* out = Ypart + (int64_t)split * p * d;
#pragma unroll
    for (int j = 0; j < PM; ++j)
      if (j < p) out[(int64_t)j * d + row] = acc[j];
  }
}

// out = alpha * sum_split Ypart + beta * A + gamma * B (fixed summation order).
__global__ __launch_bounds__(NT) void k_reduce_y(const double* __restrict__ Ypart, int nsplit,
                                                 int64_t cnt, double alpha,
                                                 const double* __restrict__ A, double beta,
                                                 const double* __restrict__ B, double gamma,
                                                 double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= cnt) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += Ypart[(int64_t)k * cnt + e];
  double v = alpha * s;
  if (A) v += beta * A[e];
  if (B) v += gamma * B[e];
  out[e] = v;
}

// ---------------------------------------------------------------------------
// Inner step, part 1.  A workgroup owns NS samples: draws them, then computes
// C[s, :] = scale_s * x_{i_s}^T Dl with 64-row slabs of the sampled columns
// and of Dl staged in LDS.
constexpr int SD_NS = 16;
template <typename TX, int PM>
__global__ __launch_bounds__(NT) void k_sample_dot(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                   int64_t n, int p,
                                                   const uint64_t* __restrict__ cdf, uint32_t k0,
                                                   uint32_t k1, uint32_t step, uint32_t epoch,
                                                   uint32_t word3, int64_t b,
                                                   const double* __restrict__ Dl,
                                                   int32_t* __restrict__ idx_out,
                                                   double* __restrict__ scale_out,
                                                   double* __restrict__ C) {
  constexpr int NQ = (PM + 15) / 16;
  __shared__ int64_t sidx[SD_NS];
  __shared__ double ssc[SD_NS];
  __shared__ double xs[64][SD_NS + 1];
  __shared__ double ds[64][PM + 1];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * SD_NS;
  if (t < SD_NS) {
    const int64_t j = s0 + t;
    if (j < b) {
      int64_t i;
      double sc;
      draw_one(cdf, n, k0, k1, (uint32_t)j, step, epoch, word3, b, &i, &sc);
      sidx[t] = i;
      ssc[t] = sc;
      idx_out[j] = (int32_t)i;
      scale_out[j] = sc;
    } else {
      sidx[t] = -1;
      ssc[t] = 0.0;
    }
  }
  __syncthreads();
  const int s = t % SD_NS, jg = t / SD_NS;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t r0 = 0; r0 < d; r0 += 64) {
    for (int e = t; e < 64 * SD_NS; e += NT) {
      const int rr = e % 64, ss = e / 64;
      const int64_t r = r0 + rr;
      const int64_t ci = sidx[ss];
      xs[rr][ss] = (r < d && ci >= 0) ? ldx(X, ci * ld + r) : 0.0;
    }
    for (int e = t; e < 64 * PM; e += NT) {
      const int rr = e % 64, jj = e / 64;
      const int64_t r = r0 + rr;
      ds[rr][jj] = (r < d && jj < p) ? Dl[(int64_t)jj * d + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 64; ++rr) {
      const double xv = xs[rr][s];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = jg + 16 * q;
        if (j < PM) acc[q] = fma(xv, ds[rr][j], acc[q]);
      }
    }
    __syncthreads();
  }
  if (s0 + s < b) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = jg + 16 * q;
      if (j < p) C[(s0 + s) * p + j] = acc[q] * ssc[s];
    }
  }
}

// Inner step, part 2.  A workgroup owns 16 rows of Dl and sums
// X[rows, i_s] C[s, :] over all b samples, 64 samples at a time through LDS.
constexpr int UP_RT = 16;
template <typename TX, int PM>
__global__ __launch_bounds__(NT) void k_update(const TX* __restrict__ X, int64_t ld, int64_t d,
                                               int p, int64_t b, const int32_t* __restrict__ idx,
                                               const double* __restrict__ C,
                                               const double* __restrict__ G,
                                               double* __restrict__ Dl, double lam, double eta) {
  constexpr int NQ = (PM + 15) / 16;
  __shared__ double xs[64][UP_RT + 1];
  __shared__ double cs[64][PM + 1];
  const int t = threadIdx.x;
  const int r = t % UP_RT, jg = t / UP_RT;
  const int64_t r0 = (int64_t)blockIdx.x * UP_RT;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t s0 = 0; s0 < b; s0 += 64) {
    for (int e = t; e < 64 * UP_RT; e += NT) {
      const int ss = e / UP_RT, rr = e % UP_RT;
      const int64_t s = s0 + ss, row = r0 + rr;
      xs[ss][rr] = (s < b && row < d) ? ldx(X, (int64_t)idx[s] * ld + row) : 0.0;
    }
    for (int e = t; e < 64 * PM; e += NT) {
      const int ss = e / PM, jj = e % PM;
      const int64_t s = s0 + ss;
      cs[ss][jj] = (s < b && jj < p) ? C[s * p + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ss = 0; ss < 64; ++ss) {
      const double xv = xs[ss][r];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int j = jg + 16 * q;
        if (j < PM) acc[q] = fma(xv, cs[ss][j], acc[q]);
      }
    }
    __syncthreads();
  }
  const int64_t row = r0 + r;
  if (row < d) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int j = jg + 16 * q;
      if (j < p) {
        const int64_t e = (int64_t)j * d + row;
        const double dl = Dl[e];
        Dl[e] = dl - eta * (G[e] + lam * dl - acc[q]);
      }
    }
  }
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

// D = A M + beta C ; one thread per row, M in LDS.
template <int PM>
__global__ __launch_bounds__(NT) void k_gemm_small(int64_t d, int p, int q,
                                                   const double* __restrict__ A,
                                                   const double* __restrict__ M, int ldm,
                                                   double* __restrict__ D, double beta,
                                                   const double* __restrict__ C) {
  __shared__ double ms[64 * 64];
  const int t = threadIdx.x;
  for (int e = t; e < p * q; e += NT) ms[e] = M[(e % p) + (int64_t)(e / p) * ldm];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * NT + t;
  if (row >= d) return;
  double acc[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) acc[j] = 0.0;
  for (int i = 0; i < p; ++i) {
    const double a = A[(int64_t)i * d + row];
#pragma unroll
    for (int j = 0; j < PM; ++j)
      if (j < q) acc[j] = fma(a, ms[i + j * p], acc[j]);
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

__global__ __launch_bounds__(NT) void k_chol_rinv(const double* __restrict__ G, int m,
                                                  double* __restrict__ Rinv,
                                                  int* __restrict__ info) {
  __shared__ double a[SM][SM];
  __shared__ double li[SM][SM];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < m * m; e += NT) {
    const int i = e % m, j = e / m;
    a[i][j] = 0.5 * (G[i + j * m] + G[j + i * m]);
  }
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (t == 0) {
      const double dj = a[j][j];
      if (!(dj > 0.0) || !isfinite(dj)) {
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
  __shared__ double a[SM][SM];
  __shared__ double v[SM][SM];
  __shared__ double rc[SM / 2], rs[SM / 2];
  __shared__ int rp[SM / 2], rq[SM / 2];
  __shared__ double red[NT];
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
    double off = 0.0, tot = 0.0;
    for (int e = t; e < m * m; e += NT) {
      const int i = e % m, j = e / m;
      const double x = a[i][j] * a[i][j];
      tot += x;
      if (i != j) off += x;
    }
    red[t] = off;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
      if (t < k) red[t] += red[t + k];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[t] = tot;
    __syncthreads();
    for (int k = NT / 2; k > 0; k >>= 1) {
      if (t < k) red[t] += red[t + k];
      __syncthreads();
    }
    if (t == 0) stop = (offs <= 1e-32 * red[0]) || m < 2;
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
          a[row][P] = c * aP - s * aQ;
          a[row][Q] = s * aP + c * aQ;
          const double vP = v[row][P], vQ = v[row][Q];
          v[row][P] = c * vP - s * vQ;
          v[row][Q] = s * vP + c * vQ;
        }
      }
      __syncthreads();
      if (t < np && rp[t] >= 0 && rs[t] != 0.0) {
        a[rp[t]][rq[t]] = 0.0;
        a[rq[t]][rp[t]] = 0.0;
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

__global__ __launch_bounds__(NT) void k_sign_fix(double* __restrict__ U, int64_t d) {
  __shared__ double bv[NT];
  __shared__ int64_t bi[NT];
  const int t = threadIdx.x;
  double* col = U + (int64_t)blockIdx.x * d;
  double best = -1.0;
  int64_t am = 0;
  for (int64_t r = t; r < d; r += NT) {
    const double x = fabs(col[r]);
    if (x > best) {
      best = x;
      am = r;
    }
  }
  bv[t] = best;
  bi[t] = am;
  __syncthreads();
  for (int k = NT / 2; k > 0; k >>= 1) {
    if (t < k) {
      const double o = bv[t + k];
      const int64_t oi = bi[t + k];
      if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
        bv[t] = o;
        bi[t] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = col[bi[0]] < 0.0 ? -1.0 : 1.0;
  for (int64_t r = t; r < d; r += NT) col[r] *= sg;
}

inline unsigned nblocks(int64_t count, int per = NT) {
  return (unsigned)((count + per - 1) / per);
}

}  // namespace

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
                 k_colnorm<TX><<<nblocks(X.n), NT, 0, st>>>((const TX*)X.v, X.ld, X.d, X.n, w,
                                                            bad));
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

int pass_nsplit(int64_t d, int64_t n) {
  const int64_t rowtiles = (d + NT - 1) / NT;
  int64_t ns = (1024 + rowtiles - 1) / rowtiles;
  const int64_t maxs = (n + 63) / 64;
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return (int)ns;
}

hipError_t pass_xtw(const XView& X, const double* W, int p, double* T, hipStream_t st) {
  LR_DISPATCH_DT(X.dt, TX,
                 LR_DISPATCH_PM(p, PM,
                                k_xtw<TX, PM><<<nblocks(X.n), NT, 0, st>>>(
                                    (const TX*)X.v, X.ld, X.d, X.n, p, W, T)));
  return hipGetLastError();
}

hipError_t pass_xt(const XView& X, const double* T, int p, const PassBufs& pb, double alpha,
                   const double* A, double beta, const double* B, double gamma, double* out,
                   hipStream_t st) {
  const int64_t cps = (X.n + pb.nsplit - 1) / pb.nsplit;
  dim3 grid(nblocks(X.d), (unsigned)pb.nsplit);
  LR_DISPATCH_DT(X.dt, TX,
                 LR_DISPATCH_PM(p, PM,
                                k_xt<TX, PM><<<grid, NT, 0, st>>>((const TX*)X.v, X.ld, X.d, X.n,
                                                                  p, T, cps, pb.Ypart)));
  const int64_t cnt = X.d * p;
  k_reduce_y<<<nblocks(cnt), NT, 0, st>>>(pb.Ypart, pb.nsplit, cnt, alpha, A, beta, B, gamma, out);
  return hipGetLastError();
}

hipError_t step_sample_dot(const XView& X, int p, const uint64_t* cdf, uint64_t seed,
                           uint32_t step, uint32_t epoch, uint32_t word3, int64_t b,
                           const double* Dl, int32_t* idx, double* scale, double* C,
                           hipStream_t st) {
  const unsigned grid = nblocks(b, SD_NS);
  LR_DISPATCH_DT(X.dt, TX,
                 LR_DISPATCH_PM(p, PM,
                                k_sample_dot<TX, PM><<<grid, NT, 0, st>>>(
                                    (const TX*)X.v, X.ld, X.d, X.n, p, cdf, (uint32_t)seed,
                                    (uint32_t)(seed >> 32), step, epoch, word3, b, Dl, idx,
                                    scale, C)));
  return hipGetLastError();
}

hipError_t step_update(const XView& X, int p, int64_t b, const int32_t* idx, const double* C,
                       const double* G, double* Dl, double lam, double eta, hipStream_t st) {
  const unsigned grid = nblocks(X.d, UP_RT);
  LR_DISPATCH_DT(X.dt, TX,
                 LR_DISPATCH_PM(p, PM,
                                k_update<TX, PM><<<grid, NT, 0, st>>>((const TX*)X.v, X.ld, X.d,
                                                                      p, b, idx, C, G, Dl, lam,
                                                                      eta)));
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

hipError_t sign_fix(double* U, int64_t d, int k, hipStream_t st) {
  k_sign_fix<<<k, NT, 0, st>>>(U, d);
  return hipGetLastError();
}

}  // namespace lr
