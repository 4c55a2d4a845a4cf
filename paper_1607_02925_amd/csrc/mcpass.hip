// Matrix-core full-gradient pass (Section 2.3: the full gradient of each SVRG
// epoch, lambda W~ - X (X^T W~) - S) for dense FP32 and BF16 X on gfx950.
//
// Two kernels, each streaming X once:
//   k_mc_xtw  T = X^T W.  Each wave owns 16 MT columns and runs over all rows;
//             lane l = 16 q + c supplies rows 8 q .. 8 q + 7 of column c of a
//             32-row block as the A operand (one 16- or 32-byte load), the
//             B operand is the W part tile of that row block, staged in LDS
//             once per workgroup.  T leaves as three BF16 parts in the B-operand
//             order of the second kernel (contraction over columns).
//   k_mc_xt   partial X T for 128 rows and one column range.  A 128 x 32 tile
//             of X is read column by column (coalesced), written to LDS
//             transposed, and each lane reads 8 consecutive columns of its row
//             as the A operand; T's part tiles of the block come through LDS.
// v_mfma_f32_16x16x32_bf16: lane l supplies row l % 16 of A and column l % 16
// of B over k = 8 (l / 16) .. + 7 and receives D[4 (l / 16) + v][l % 16].
#include "mcpass.h"

#include <hip/hip_ext.h>

#include <algorithm>

namespace lr {
namespace {

__device__ __forceinline__ int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int NW = 8;          // waves per workgroup
constexpr int NPART = 3;       // BF16 parts of W, T and FP32 X
constexpr int FLUSH = 8;       // 32-term blocks between FP32 -> FP64 flushes
constexpr int RB = NW * 16;    // rows per k_mc_xt workgroup

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Offset of (k, j) in the B-operand tile order: per block of 32 k and slice of
// 16 columns a contiguous tile of 512 values, lane 16 q + c holding k = 8 q ..
// 8 q + 7 of column c.
__device__ __forceinline__ int64_t bt_off(int64_t k, int j, int NS) {
  const int w = (int)(k & 31);
  return (((k >> 5) * NS + (j >> 4)) * 64 + (w >> 3) * 16 + (j & 15)) * 8 + (w & 7);
}

// Three BF16 parts of a double: hi, mid, lo with x - hi - mid - lo below 2^-24 |x|.
__device__ __forceinline__ void split3(double x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)(float)x;
  double r = x - (double)(float)h;
  m = (__bf16)(float)r;
  r -= (double)(float)m;
  l = (__bf16)(float)r;
}

// Parts of eight FP32 values (exact: 8 + 8 + 8 significant bits).
template <int NPX>
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8 (&o)[NPX]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float r = x[i];
#pragma unroll
    for (int g = 0; g < NPX; ++g) {
      const __bf16 h = (__bf16)r;
      o[g][i] = h;
      r -= (float)h;
    }
  }
}

template <typename TX>
struct XTraits;
template <>
struct XTraits<float> {
  static constexpr int NPX = 3, NV = 2;   // parts, 16-byte loads per 8 values
};
template <>
struct XTraits<uint16_t> {
  static constexpr int NPX = 1, NV = 1;
};

// The A operand parts of eight values held as NV 16-byte words.
template <typename TX>
__device__ __forceinline__ void a_parts(const u32x4 (&v)[XTraits<TX>::NV],
                                        bf16x8 (&o)[XTraits<TX>::NPX]) {
  if constexpr (sizeof(TX) == 2) {
    o[0] = __builtin_bit_cast(bf16x8, v[0]);
  } else {
    float x[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = __uint_as_float(v[0][i]);
      x[4 + i] = __uint_as_float(v[1][i]);
    }
    split8<3>(x, o);
  }
}

// Eight consecutive values p[r .. r + 7] of a column of d values.  Every load
// reads an in-bounds address and none sits behind a branch, so a stage's loads
// stay in flight until its data is used: VEC (d % 8 == 0, 16-byte aligned
// chunks) moves a chunk that would pass d back to rows d - 8 .. d - 1, the
// scalar form clamps each row to d - 1.  The values of rows past d are thus
// some finite entries of X; every caller multiplies them by zero parts or
// drops their results.
template <typename TX, bool VEC>
__device__ __forceinline__ void load8(const TX* __restrict__ col, int64_t r, int64_t d,
                                      u32x4 (&v)[XTraits<TX>::NV]) {
  if constexpr (VEC) {
    const u32x4* a = reinterpret_cast<const u32x4*>(col + (r + 8 <= d ? r : d - 8));
#pragma unroll
    for (int i = 0; i < XTraits<TX>::NV; ++i) v[i] = __builtin_nontemporal_load(a + i);
  } else if constexpr (sizeof(TX) == 2) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      w[h] = (uint32_t)col[imin(r + 2 * h, d - 1)] | ((uint32_t)col[imin(r + 2 * h + 1, d - 1)] << 16);
    v[0] = u32x4{w[0], w[1], w[2], w[3]};
  } else {
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = __float_as_uint(col[imin(r + i, d - 1)]);
    v[0] = u32x4{w[0], w[1], w[2], w[3]};
    v[1] = u32x4{w[4], w[5], w[6], w[7]};
  }
}

// W (d x p FP64, column-major) -> three BF16 parts in the B-operand order over
// rows (k = row), zero past d and p.
__global__ __launch_bounds__(256) void k_mc_split_w(const double* __restrict__ W, int64_t d,
                                                    int p, int PC, int64_t rows,
                                                    uint16_t* __restrict__ Wp,
                                                    int64_t wstride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * PC) return;
  const int64_t r = e / PC;
  const int j = (int)(e % PC);
  const double x = (r < d && j < p) ? W[(int64_t)j * d + r] : 0.0;
  __bf16 h, m, l;
  split3(x, h, m, l);
  const int64_t o = bt_off(r, j, PC / 16);
  __bf16* out = reinterpret_cast<__bf16*>(Wp);
  out[o] = h;
  out[wstride + o] = m;
  out[2 * wstride + o] = l;
}

// T = X^T W.  A workgroup takes one group of 128 columns; wave w owns columns
// 16 w .. 16 w + 15 and runs over all 32-row blocks.  X is fetched PD blocks
// ahead in registers; the W part tiles of the next block are staged in the
// other LDS buffer, one barrier per block.  The main loop's steps are
// unconditional and it stores nothing to memory, so each step waits only for
// the loads of its own block.
template <typename TX, int NTW, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_mc_xtw(const TX* __restrict__ X, int64_t ld,
                                                    int64_t d, int64_t n,
                                                    const uint16_t* __restrict__ Wp,
                                                    int64_t wstride, uint16_t* __restrict__ Tp,
                                                    int64_t tstride, int64_t tcols) {
  using XT = XTraits<TX>;
  constexpr int NPX = XT::NPX, NV = XT::NV;
  constexpr int PD = 3, NSTG = PD + 1;           // blocks in flight, register stages
  constexpr int TILES = NPART * NTW;             // W part tiles per row block
  constexpr int WPT = (TILES * 64 + NW * 64 - 1) / (NW * 64);   // 16-byte words per thread
  __shared__ u32x4 wsh[2][WPT * NW * 64];   // words past TILES * 64 are never read
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = NTW;
  const int64_t g0 = blockIdx.x;
  const int64_t nkb = (d + 31) / 32, total = nkb;
  auto w_word = [&](int64_t kb, int e) -> u32x4 {
    e = e < TILES * 64 ? e : TILES * 64 - 1;
    const int tile = e / 64, g = tile / NTW, u = tile % NTW;
    return *reinterpret_cast<const u32x4*>(Wp + g * wstride + ((kb * NS + u) * 64 + e % 64) * 8);
  };
  // X chunk of row block i; blocks past the end re-read the last one
  const TX* __restrict__ xcol = X + imin(g0 * 128 + 16 * wave + li, n - 1) * ld;
  auto load_x = [&](u32x4 (&xs)[NV], int64_t i) {
    load8<TX, VEC>(xcol, imin(i, total - 1) * 32 + 8 * q, d, xs);
  };
  f32x4 acc[NTW];
  double accd[NTW][4];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) accd[u][v] = 0.0;
  }
  auto compute = [&](const u32x4 (&xs)[NV], const u32x4* __restrict__ wb) {
    bf16x8 xp[NPX];
    a_parts<TX>(xs, xp);
#pragma unroll
    for (int g = 0; g < NPART; ++g)
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const bf16x8 wf = __builtin_bit_cast(bf16x8, wb[(g * NTW + u) * 64 + l]);
#pragma unroll
        for (int h = 0; h < NPX; ++h)
          if (h + g < NPART) acc[u] = mfma(xp[h], wf, acc[u]);
      }
  };
  auto flush = [&]() {
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[u][v] += (double)acc[u][v];
      acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  // lane 16 q + c holds T[16 w + 4 q + v][16 u + c] of the group; lanes with
  // even q take their partner's four rows and store eight consecutive columns
  // of T (one 16-byte word per part), zero past n
  __bf16* tout = reinterpret_cast<__bf16*>(Tp);
  auto store_t = [&](int64_t g) {
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
      double v8[8];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        v8[v] = accd[u][v];
        v8[4 + v] = __shfl_down(accd[u][v], 16);
        accd[u][v] = 0.0;
      }
      const int64_t ca = g * 128 + 16 * wave + 4 * q;
      if ((q & 1) == 0 && ca < tcols) {
        bf16x8 o[NPART];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          __bf16 h, md, lo;
          split3(ca + i < n ? v8[i] : 0.0, h, md, lo);
          o[0][i] = h;
          o[1][i] = md;
          o[2][i] = lo;
        }
        const int64_t off = bt_off(ca, 16 * u + li, NS);
#pragma unroll
        for (int g2 = 0; g2 < NPART; ++g2)
          *reinterpret_cast<bf16x8*>(tout + g2 * tstride + off) = o[g2];
      }
    }
  };
  // W words of block i + 2 are fetched at step i into wr[i & 1] and staged in
  // LDS at step i + 1, so their latency is hidden behind a whole step as well
  u32x4 xs[NSTG][NV];
  u32x4 wr[2][WPT];
  auto step = [&](int64_t i, u32x4 (&cur)[NV], u32x4 (&ahead)[NV], u32x4 (&wload)[WPT],
                  const u32x4 (&wstore)[WPT]) {
#pragma unroll
    for (int j = 0; j < WPT; ++j) wload[j] = w_word(imin(i + 2, nkb - 1), t + j * NW * 64);
    load_x(ahead, i + PD);
    compute(cur, wsh[i & 1]);
    if ((i + 1) % FLUSH == 0) flush();
#pragma unroll
    for (int j = 0; j < WPT; ++j) wsh[(i + 1) & 1][t + j * NW * 64] = wstore[j];
    __syncthreads();
  };
  for (int e = t; e < TILES * 64; e += NW * 64) wsh[0][e] = w_word(0, e);
#pragma unroll
  for (int j = 0; j < WPT; ++j) wr[1][j] = w_word(imin(1, nkb - 1), t + j * NW * 64);
#pragma unroll
  for (int j = 0; j < PD; ++j) load_x(xs[j], j);
  __syncthreads();
  int64_t i = 0;
  for (; i + NSTG <= total; i += NSTG) {
    step(i, xs[0], xs[3], wr[0], wr[1]);
    step(i + 1, xs[1], xs[0], wr[1], wr[0]);
    step(i + 2, xs[2], xs[1], wr[0], wr[1]);
    step(i + 3, xs[3], xs[2], wr[1], wr[0]);
  }
  if (i < total) step(i, xs[0], xs[3], wr[0], wr[1]);
  if (i + 1 < total) step(i + 1, xs[1], xs[0], wr[1], wr[0]);
  if (i + 2 < total) step(i + 2, xs[2], xs[1], wr[0], wr[1]);
  flush();
  store_t(g0);
}

// Partial sums of X T over the columns of split s for rows r0 .. r0 + 127;
// workgroup -> (split, row block) keeps every row block of a split on one XCD
// so the split's T tiles are fetched into one L2.  Each thread fetches one
// column's 8-row chunk of the next-but-one 32-column block and its share of
// the T part tiles; a block is staged (X transposed) in the other LDS buffer
// while the current one is multiplied, one barrier per block.
// part: row-major rows x PC.
template <typename TX, int NTW, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_mc_xt(const TX* __restrict__ X, int64_t ld, int64_t d,
                                                   int64_t n, const uint16_t* __restrict__ Tp,
                                                   int64_t tstride, int nrb, int64_t kper,
                                                   float* __restrict__ part, int64_t pstride) {
  using XT = XTraits<TX>;
  constexpr int NPX = XT::NPX, NV = XT::NV;
  constexpr int TT = NPART * NTW;                      // T part tiles per column block
  constexpr int TPT = (TT * 64 + NW * 64 - 1) / (NW * 64);
  constexpr int LDP = sizeof(TX) == 4 ? 33 : 34;       // LDS row pitch (elements)
  __shared__ TX xs[2][RB * LDP];
  __shared__ u32x4 ts[2][TPT * NW * 64];   // words past TT * 64 are never read
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = NTW;
  const int id = blockIdx.x, loc = id / 8;
  const int64_t s = (int64_t)(loc / nrb) * 8 + id % 8;
  const int64_t r0 = (int64_t)(loc % nrb) * RB;
  const int64_t kb0 = s * kper / 32;
  const int64_t kb1 = imin((s + 1) * kper, (n + 31) / 32 * 32) / 32;
  // loader: column cc of the block, rows rr .. rr + 7 of the row block
  const int cc = t / 16, rr = (t % 16) * 8;
  struct Stage {
    u32x4 x[NV];
    u32x4 tw[TPT];
  };
  auto load = [&](Stage& S, int64_t kb) {
    kb = imin(kb, kb1 - 1);
    const int64_t col = imin(kb * 32 + cc, n - 1);
    load8<TX, VEC>(X + col * ld, r0 + rr, d, S.x);
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      int e = t + i * NW * 64;
      e = e < TT * 64 ? e : TT * 64 - 1;
      const int tile = e / 64, g = tile / NTW, u = tile % NTW;
      S.tw[i] = *reinterpret_cast<const u32x4*>(Tp + g * tstride +
                                                ((kb * NS + u) * 64 + e % 64) * 8);
    }
  };
  auto stage_lds = [&](const Stage& S, int buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (sizeof(TX) == 4)
        xs[buf][(rr + i) * LDP + cc] = __uint_as_float(S.x[i / 4][i % 4]);
      else
        xs[buf][(rr + i) * LDP + cc] = (uint16_t)(S.x[0][i / 2] >> (16 * (i % 2)));
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) ts[buf][t + i * NW * 64] = S.tw[i];
  };
  f32x4 acc[NTW];
  double accd[NTW][4];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) accd[u][v] = 0.0;
  }
  const int arow = (wave * 16 + li) * LDP + 8 * q;
  auto compute = [&](int buf) {
    u32x4 av[NV];
    if constexpr (sizeof(TX) == 4) {
      const uint32_t* xw = reinterpret_cast<const uint32_t*>(xs[buf]) + arow;
      av[0] = u32x4{xw[0], xw[1], xw[2], xw[3]};
      av[1] = u32x4{xw[4], xw[5], xw[6], xw[7]};
    } else {
      const uint32_t* xw = reinterpret_cast<const uint32_t*>(xs[buf]) + arow / 2;
      av[0] = u32x4{xw[0], xw[1], xw[2], xw[3]};
    }
    bf16x8 xp[NPX];
    a_parts<TX>(av, xp);
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int g = 0; g < NPART; ++g) {
        const bf16x8 tb = __builtin_bit_cast(bf16x8, ts[buf][(g * NTW + u) * 64 + l]);
#pragma unroll
        for (int h = 0; h < NPX; ++h)
          if (h + g < NPART) acc[u] = mfma(xp[h], tb, acc[u]);
      }
  };
  auto flush = [&]() {
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[u][v] += (double)acc[u][v];
      acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  // block kb + 1 goes to LDS (its loads were issued two blocks earlier) and its
  // registers are refilled with block kb + 3 while block kb is multiplied
  auto step = [&](int64_t kb, Stage& nxt) {
    stage_lds(nxt, (int)((kb + 1) & 1));
    load(nxt, kb + 3);
    compute((int)(kb & 1));
    if ((kb - kb0 + 1) % FLUSH == 0) flush();
    __syncthreads();
  };
  if (kb0 < kb1) {
    Stage A, B;
    load(A, kb0);
    load(B, kb0 + 1);
    stage_lds(A, (int)(kb0 & 1));
    load(A, kb0 + 2);
    __syncthreads();
    int64_t kb = kb0;
    for (; kb + 2 <= kb1; kb += 2) {
      step(kb, B);
      step(kb + 1, A);
    }
    if (kb < kb1) step(kb, B);
    flush();
  }
  // lane 16 q + c holds rows 4 q + v of the wave's 16, column 16 u + c
  float* __restrict__ out = part + s * pstride;
#pragma unroll
  for (int u = 0; u < NTW; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = r0 + wave * 16 + 4 * q + v;
      out[r * (NTW * 16) + 16 * u + li] = (float)accd[u][v];
    }
}

// out[j d + r] = alpha sum_s part[s][r PC + j] + beta A + gamma B, the splits
// added in order in FP64.
__global__ __launch_bounds__(256) void k_mc_reduce(const float* __restrict__ part, int nsplit,
                                                   int64_t pstride, int64_t d, int p, int PC,
                                                   double alpha, const double* __restrict__ A,
                                                   double beta, const double* __restrict__ B,
                                                   double gamma, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= d * p) return;
  const int64_t r = e / p;
  const int j = (int)(e % p);
  double sum = 0.0;
  for (int s = 0; s < nsplit; ++s) sum += (double)part[s * pstride + r * PC + j];
  const int64_t o = (int64_t)j * d + r;
  double v = alpha * sum;
  if (A) v += beta * A[o];
  if (B) v += gamma * B[o];
  out[o] = v;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Split {
  int nrb, nsplit;
  int64_t kper;
};

Split mc_split(int64_t d, int64_t n) {
  Split sp;
  sp.nrb = (int)((d + RB - 1) / RB);
  // about 1024 workgroups; a multiple of 8 splits for the XCD mapping
  int64_t ns = round_up(std::max<int64_t>(8, (1024 + sp.nrb - 1) / sp.nrb), 8);
  ns = std::min<int64_t>(ns, round_up((n + 31) / 32, 8));
  sp.kper = round_up((n + ns - 1) / ns, 32);
  sp.nsplit = (int)ns;
  return sp;
}

template <typename K, typename... Args>
void launch_mc(K kernel, dim3 grid, dim3 block, hipStream_t st, const Probe& pr, Args... args) {
  if (pr.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pr.start, pr.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

}  // namespace

McSizes mc_sizes(int64_t d, int64_t n, int PC) {
  const Split sp = mc_split(d, n);
  McSizes z;
  z.nsplit = sp.nsplit;
  z.wp_elems = (int64_t)NPART * round_up(d, 32) * PC;
  z.tp_elems = (int64_t)NPART * round_up(n, 32) * PC;
  z.part_elems = (int64_t)sp.nsplit * sp.nrb * RB * PC;
  return z;
}

#define MC_DISPATCH_NTW(nt, NTW, ...) \
  switch (nt) {                       \
    case 1: {                         \
      constexpr int NTW = 1;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 2: {                         \
      constexpr int NTW = 2;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 3: {                         \
      constexpr int NTW = 3;          \
      __VA_ARGS__;                    \
    } break;                          \
    case 4: {                         \
      constexpr int NTW = 4;          \
      __VA_ARGS__;                    \
    } break;                          \
    default:                          \
      return hipErrorInvalidValue;    \
  }

hipError_t mc_pass(const XView& X, const double* W, int p, int PC, const McBufs& mb,
                   double alpha, const double* A, double beta, const double* B, double gamma,
                   double* out, hipStream_t st, const Probe& pr, const Probe& pr2) {
  if ((X.dt != 1 && X.dt != 2) || X.ld % 8 || (uintptr_t)X.v % 16 || PC % 16 || PC > 64 ||
      p < 1 || p > PC || X.d < 1 || X.n < 1)
    return hipErrorInvalidValue;
  const Split sp = mc_split(X.d, X.n);
  const int64_t wstride = round_up(X.d, 32) * PC, tstride = round_up(X.n, 32) * PC;
  if (sp.nsplit != mb.nsplit || wstride != mb.wstride || tstride != mb.tstride)
    return hipErrorInvalidValue;
  const int64_t pstride = (int64_t)sp.nrb * RB * PC;
  const int64_t wrows = round_up(X.d, 32);
  k_mc_split_w<<<(unsigned)((wrows * PC + 255) / 256), 256, 0, st>>>(W, X.d, p, PC, wrows, mb.Wp,
                                                                     wstride);
  const int64_t tcols = round_up(X.n, 32);
  const bool vec = X.d % 8 == 0 && X.d >= 8;
  const dim3 g1((unsigned)((X.n + 127) / 128));
  const dim3 g2((unsigned)(sp.nrb * sp.nsplit));
#define MC_LAUNCH(TX, NTW, VEC)                                                              \
  do {                                                                                       \
    launch_mc(k_mc_xtw<TX, NTW, VEC>, g1, dim3(NW * 64), st, pr, (const TX*)X.v, X.ld, X.d, \
              X.n, mb.Wp, wstride, mb.Tp, tstride, tcols);                                   \
    launch_mc(k_mc_xt<TX, NTW, VEC>, g2, dim3(NW * 64), st, pr2, (const TX*)X.v, X.ld, X.d, \
              X.n, mb.Tp, tstride, sp.nrb, sp.kper, mb.part, pstride);                       \
  } while (0)
  MC_DISPATCH_NTW(PC / 16, NTW, {
    if (X.dt == 1) {
      if (vec) MC_LAUNCH(float, NTW, true);
      else MC_LAUNCH(float, NTW, false);
    } else {
      if (vec) MC_LAUNCH(uint16_t, NTW, true);
      else MC_LAUNCH(uint16_t, NTW, false);
    }
  });
#undef MC_LAUNCH
  k_mc_reduce<<<(unsigned)((X.d * p + 255) / 256), 256, 0, st>>>(
      mb.part, sp.nsplit, pstride, X.d, p, PC, alpha, A, beta, B, gamma, out);
  return hipGetLastError();
}

}  // namespace lr
