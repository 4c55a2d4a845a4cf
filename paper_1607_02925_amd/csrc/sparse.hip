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
// heavy row serialises the pass).  The inner-step update adds into the rows
// of its b sampled columns in a fixed order: the contributions are sorted by
// row and each row's run is summed in sample order (csc_step_scatter_sorted).
// Where the b x (largest column) contributions would not fit the plan's cap,
// the update falls back to FP64 atomics (the rows that occur most often summed
// per workgroup in LDS first), whose rounding order depends on timing.
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

// The inner-step scatter in a fixed order.  Contribution t = j maxnnz + kk
// (sample j, the kk-th stored entry of column idx[j]) adds eta v_k C[j, :] to
// row ri[k], k = cp[idx[j]] + kk.  The contributions are sorted by row with a
// stable radix sort (positions whose kk is past the column's entries carry the
// key `pad` >= d and sort last), so each row's contributions form one run in
// ascending t.  Each wave sums the runs of SG_CH consecutive sorted
// contributions in that order; a run wholly inside the chunk is added to its
// row directly (no other wave touches that row), a run that crosses a chunk
// boundary leaves its pieces in `carry`, and the workgroup of the chunk where
// the run starts adds them up in a fixed order.  Nothing depends on timing.
constexpr int SG_CH = 64;       // sorted contributions per wave
constexpr int SG_WAVES = 4;     // waves per workgroup of k_sp_runs
constexpr int SG_PREV = 1;      // the chunk's first run began in an earlier chunk
constexpr int SG_NEXT = 2;      // the chunk's last run goes on into the next chunk
constexpr int SG_SINGLE = 4;    // the chunk holds one run only

template <typename TX>
__global__ __launch_bounds__(NT) void k_sp_keys(const TX* __restrict__ v,
                                                const int32_t* __restrict__ cp,
                                                const int32_t* __restrict__ ri,
                                                const int32_t* __restrict__ idx, int64_t total,
                                                int maxnnz, uint32_t pad,
                                                uint32_t* __restrict__ keys,
                                                int32_t* __restrict__ pos,
                                                double* __restrict__ xval) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= total) return;
  const int64_t j = t / maxnnz;
  const int64_t i = idx[j];
  const int64_t k = cp[i] + (t - j * maxnnz);
  const bool in = k < cp[i + 1];
  keys[t] = in ? (uint32_t)ri[k] : pad;
  xval[t] = in ? ldv(v, k) : 0.0;
  pos[t] = (int32_t)t;
}

// Stable least-significant-digit radix sort of (key, position) pairs, 8 bits
// per pass, in three kernels per pass: digit counts per tile of RS_TILE items;
// per digit, the exclusive prefix of its counts over the tiles and its total;
// and a scatter in which each tile starts digit g at (sum of the totals of the
// digits below g) + (its prefix of g) and ranks its items in index order
// (within a wave by matching the digit across lanes, across the tile's waves
// and rounds by counters in LDS).  Integer work only: the order is exact and
// does not depend on timing.
constexpr int RS_T = 256, RS_IPT = 8, RS_TILE = RS_T * RS_IPT, RS_W = RS_T / 64;
constexpr int RS_SCAN_T = 1024, RS_SCAN_PT = 2;   // tiles per thread in k_rs_scan
constexpr int64_t RS_MAX_TILES = (int64_t)RS_SCAN_T * RS_SCAN_PT;

__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t N,
                                                  int shift, int64_t ntiles,
                                                  int32_t* __restrict__ hist) {
  __shared__ int32_t cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_IPT; ++r) {
    const int64_t e = base + r * RS_T + t;
    if (e < N) atomicAdd(&cnt[(keys[e] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)t * ntiles + blockIdx.x] = cnt[t];
}

// Digit blockIdx.x: its counts over the tiles (hist row) become their exclusive
// prefix, and its total goes to tot[digit].  ntiles <= RS_MAX_TILES.
__global__ __launch_bounds__(RS_SCAN_T) void k_rs_scan(int32_t* __restrict__ hist,
                                                       int64_t ntiles,
                                                       int32_t* __restrict__ tot) {
  __shared__ int32_t part[RS_SCAN_T];
  const int t = threadIdx.x;
  int32_t* __restrict__ row = hist + (int64_t)blockIdx.x * ntiles;
  int32_t h[RS_SCAN_PT];
  int32_t s = 0;
#pragma unroll
  for (int u = 0; u < RS_SCAN_PT; ++u) {
    const int64_t i = (int64_t)t * RS_SCAN_PT + u;
    h[u] = i < ntiles ? row[i] : 0;
    s += h[u];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < RS_SCAN_T; off <<= 1) {
    const int32_t add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
#pragma unroll
  for (int u = 0; u < RS_SCAN_PT; ++u) {
    const int64_t i = (int64_t)t * RS_SCAN_PT + u;
    if (i < ntiles) row[i] = run;
    run += h[u];
  }
  if (t == RS_SCAN_T - 1) tot[blockIdx.x] = part[t];
}

__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                     const int32_t* __restrict__ vin, int64_t N,
                                                     int shift, int64_t ntiles,
                                                     const int32_t* __restrict__ offs,
                                                     const int32_t* __restrict__ tot,
                                                     uint32_t* __restrict__ kout,
                                                     int32_t* __restrict__ vout) {
  static_assert(RS_T == 256, "one thread per digit");
  __shared__ int32_t running[256];
  __shared__ int32_t wcnt[RS_W][256];
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  // where digit t of this tile starts: the totals of the digits below t (an
  // exclusive scan over the 256 totals in LDS) plus this tile's prefix of t
  const int32_t mine = offs[(int64_t)t * ntiles + blockIdx.x];
  running[t] = tot[t];
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t add = t >= off ? running[t - off] : 0;
    __syncthreads();
    running[t] += add;
    __syncthreads();
  }
  const int32_t below_digits = t > 0 ? running[t - 1] : 0;
  __syncthreads();
  running[t] = below_digits + mine;
  const uint64_t below_mask = (1ull << lane) - 1;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_IPT; ++r) {
#pragma unroll
    for (int w = 0; w < RS_W; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const int64_t e = base + r * RS_T + t;
    const bool valid = e < N;
    const uint32_t k = valid ? kin[e] : 0u;
    const int32_t v = valid ? vin[e] : 0;
    const int dg = (int)((k >> shift) & 255u);
    uint64_t peers = __ballot(valid);   // valid lanes of this wave with the same digit
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t m = __ballot((dg >> bit) & 1);
      peers &= ((dg >> bit) & 1) ? m : ~m;
    }
    const int below = __popcll(peers & below_mask);
    if (valid && below == 0) wcnt[wave][dg] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int at = running[dg] + below;
      for (int w = 0; w < wave; ++w) at += wcnt[w][dg];
      kout[at] = k;
      vout[at] = v;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < RS_W; ++w) add += wcnt[w][t];
    running[t] += add;
    __syncthreads();
  }
}

// Runs of the sorted contributions, one chunk of SG_CH per wave (lane l
// fetches contribution l of the chunk, lanes c < p then add column c of every
// contribution in order).  carry[(2 ch + 0) PC + c]: the first run's piece when
// it began in an earlier chunk; carry[(2 ch + 1) PC + c]: the last run's piece
// when it goes on into the next chunk and began in this one.
template <int PC>
__global__ __launch_bounds__(SG_WAVES * 64) void k_sp_runs(
    const uint32_t* __restrict__ keys, const int32_t* __restrict__ pos, int64_t total,
    int maxnnz, const double* __restrict__ xval, const double* __restrict__ C, int p,
    double eta, uint32_t pad, double* __restrict__ Dlrm, double* __restrict__ carry,
    int32_t* __restrict__ flags) {
  const int lane = threadIdx.x % 64;
  const int64_t ch = (int64_t)blockIdx.x * SG_WAVES + threadIdx.x / 64;
  const int64_t e0 = ch * SG_CH;
  if (e0 >= total) return;
  const int64_t e = e0 + lane;
  const uint32_t key = e < total ? keys[e] : pad;
  int jl = 0;
  double xl = 0.0;
  if (key != pad) {
    const int32_t t = pos[e];
    jl = t / maxnnz;
    xl = xval[t];
  }
  const uint32_t kprev = e0 > 0 ? keys[e0 - 1] : pad;
  const uint32_t knext = e0 + SG_CH < total ? keys[e0 + SG_CH] : pad;
  // valid contributions form a prefix of the chunk (pads sort last)
  const int nv = __popcll(__ballot(key != pad));
  const int c = lane < PC ? lane : PC - 1;
  double acc = 0.0;
  int runs = 0, fl = 0, start = 0;
  constexpr int U = 8;   // C rows fetched together
  static_assert(SG_CH % U == 0, "whole batches");
  // the loop index is the same in every lane, so lane i's values are read
  // with readlane (a scalar register) rather than a shuffle through LDS
  auto lane_u32 = [](uint32_t x, int i) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, i);
  };
  auto lane_f64 = [](double x, int i) {
    const uint64_t u = __double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, i);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), i);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  };
  // Runs that end inside the chunk and are added to Dlrm directly (not the first
  // run when it began in the previous chunk, not a run going on into the next
  // one) are known before the loop; their rows of Dlrm are fetched with each
  // batch's rows of C, so no read of Dlrm waits inside the loop.
  // (the shuffle runs in every lane: a lane left out of it would hand its
  // neighbour nothing)
  const uint32_t kdown = __shfl_down(key, 1);
  const uint32_t kn = lane < SG_CH - 1 ? kdown : knext;
  const uint64_t ends = __ballot(key != pad && kn != key);
  uint64_t direct = ends;
  if (nv > 0 && kprev == lane_u32(key, 0)) direct &= direct - 1;   // drop the first run's end
  if (nv == SG_CH && knext == lane_u32(key, SG_CH - 1)) direct &= ~(1ull << (SG_CH - 1));
  for (int i0 = 0; i0 < nv; i0 += U) {
    double cv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u)   // lanes past nv hold sample 0: an in-bounds row of C
      cv[u] = C[(int64_t)lane_u32((uint32_t)jl, i0 + u) * PC + c];
#pragma unroll
    for (int u = 0; u < U; ++u)
      dv[u] = (direct >> (i0 + u)) & 1 ? Dlrm[(int64_t)lane_u32(key, i0 + u) * PC + c] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      if (i >= nv) break;
      acc += lane_f64(xl, i) * (eta * cv[u]);
      if (!((ends >> i) & 1) && i + 1 < SG_CH) continue;
      // the run of row r ends at i
      const uint32_t r = lane_u32(key, i);
      const bool cprev = start == 0 && kprev == r;
      const bool cnext = i + 1 == SG_CH && knext == r;
      if (cprev) {
        fl |= SG_PREV;
        if (lane < PC) carry[(2 * ch) * PC + lane] = acc;
      } else if (cnext) {
        if (lane < PC) carry[(2 * ch + 1) * PC + lane] = acc;
      } else if (lane < p) {
        Dlrm[(int64_t)r * PC + lane] = dv[u] + acc;
      }
      if (cnext) fl |= SG_NEXT;
      ++runs;
      acc = 0.0;
      start = i + 1;
    }
  }
  if (runs == 1) fl |= SG_SINGLE;
  if (lane == 0) flags[ch] = fl;
}

// Runs that cross chunks: the workgroup of the chunk where such a run begins
// finds the chunk where it ends, sums the pieces (the starting chunk's last
// piece, then the later chunks' first pieces: NT / PC groups take every
// (NT / PC)-th chunk, each group in four interleaved partial sums added as
// (s0 + s1) + (s2 + s3), and the group sums are added in group order) and adds
// the total to the run's row.
template <int PC>
__global__ __launch_bounds__(NT) void k_sp_cross(const uint32_t* __restrict__ keys,
                                                 int64_t nch, const int32_t* __restrict__ flags,
                                                 const double* __restrict__ carry, int p,
                                                 double* __restrict__ Dlrm) {
  constexpr int G = NT / PC;
  __shared__ int64_t s_end;
  __shared__ double gsum[G * PC];
  const int64_t c0 = blockIdx.x;
  const int f = flags[c0];
  if (!(f & SG_NEXT) || ((f & SG_SINGLE) && (f & SG_PREV))) return;
  const int t = threadIdx.x;
  // the run goes through every chunk that holds only it and goes on again
  if (t == 0) s_end = nch;
  __syncthreads();
  for (int64_t base = c0 + 1; base < nch; base += NT) {
    const int64_t c2 = base + t;
    if (c2 < nch && (flags[c2] & (SG_SINGLE | SG_NEXT)) != (SG_SINGLE | SG_NEXT))
      atomicMin((unsigned long long*)&s_end, (unsigned long long)c2);
    __syncthreads();
    if (s_end < nch) break;
    __syncthreads();
  }
  const int64_t c1 = s_end < nch ? s_end : nch - 1;   // chunk where the run ends
  const int g = t / PC, col = t % PC;
  if (g < G) {   // NT need not be a multiple of PC
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t c2 = c0 + 1 + g;
    for (; c2 + 3 * G <= c1; c2 += 4 * G) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += carry[(2 * (c2 + u * G)) * PC + col];
    }
#pragma unroll
    for (int u = 0; u < 3; ++u, c2 += G)   // at most three left per group
      if (c2 <= c1) s4[u] += carry[(2 * c2) * PC + col];
    gsum[g * PC + col] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  }
  __syncthreads();
  if (t < p) {
    double tot = carry[(2 * c0 + 1) * PC + t];
    for (int h = 0; h < G; ++h) tot += gsum[h * PC + t];
    const uint32_t r = keys[c0 * SG_CH + SG_CH - 1];
    Dlrm[(int64_t)r * PC + t] += tot;
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

int64_t sp_chunks(int64_t total) { return (total + SG_CH - 1) / SG_CH; }

int64_t sp_sort_tiles(int64_t total) { return (total + RS_TILE - 1) / RS_TILE; }

size_t sp_sort_bytes(int64_t total_max, int PC) {
  return (size_t)total_max * 24 + (size_t)(sp_sort_tiles(total_max) + 1) * 256 * 4 +
         (size_t)sp_chunks(total_max) * (2 * PC * 8 + 4);
}

hipError_t csc_step_scatter_sorted(const CscView& X, int64_t b, int maxnnz, const int32_t* idx,
                                   const double* C, int PC, int p, double eta,
                                   const SpSortBufs& sb, double* Dlrm, hipStream_t st,
                                   const Probe& pr) {
  const int64_t total = b * (int64_t)maxnnz;
  if (p > PC || maxnnz < 1 || b < 1 || total > sb.total_max || X.d >= (int64_t)UINT32_MAX ||
      sp_sort_tiles(total) > RS_MAX_TILES)
    return hipErrorInvalidValue;
  const uint32_t pad = (uint32_t)X.d;   // above every row id, inside key_bits(d + 1)
  SP_DISPATCH_DT(X.dt, TX,
                 k_sp_keys<TX><<<blocks(total), NT, 0, st>>>((const TX*)X.v, X.cp, X.ri, idx,
                                                             total, maxnnz, pad, sb.keys_in,
                                                             sb.pos_in, sb.xval));
  // radix passes over the bits of d + 1, ping-ponging between the buffer pairs
  const int64_t ntiles = sp_sort_tiles(total);
  uint32_t *ka = sb.keys_in, *kb = sb.keys_out;
  int32_t *pa = sb.pos_in, *pb = sb.pos_out;
  for (int shift = 0; shift < key_bits(X.d + 1); shift += 8) {
    k_rs_hist<<<(unsigned)ntiles, RS_T, 0, st>>>(ka, total, shift, ntiles, sb.hist);
    k_rs_scan<<<256, RS_SCAN_T, 0, st>>>(sb.hist, ntiles, sb.hist + 256 * ntiles);
    k_rs_scatter<<<(unsigned)ntiles, RS_T, 0, st>>>(ka, pa, total, shift, ntiles, sb.hist,
                                                    sb.hist + 256 * ntiles, kb, pb);
    std::swap(ka, kb);
    std::swap(pa, pb);
  }
  const int64_t nch = sp_chunks(total);
  SP_DISPATCH_PC(PC, PCT, {
    launch_sp(k_sp_runs<PCT>, dim3((unsigned)((nch + SG_WAVES - 1) / SG_WAVES)),
              dim3(SG_WAVES * 64), st, pr, (const uint32_t*)ka, (const int32_t*)pa, total, maxnnz,
              (const double*)sb.xval, C, p, eta, pad, Dlrm, sb.carry, sb.flags);
    k_sp_cross<PCT><<<(unsigned)nch, NT, 0, st>>>(ka, nch, sb.flags, sb.carry, p, Dlrm);
  });
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
