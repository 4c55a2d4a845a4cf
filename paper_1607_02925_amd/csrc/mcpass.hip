// Matrix-core full-gradient pass (Section 2.3: the full gradient of each SVRG
// epoch, lambda W~ - X (X^T W~) - S) for dense FP32 and BF16 X on gfx950.
//
// Two kernels, each streaming X once:
//   k_mc_xtw  T = X^T W for 128 columns per workgroup (a 16-column tile per
//             wave) over all rows, in 64-row stages staged through LDS; lane
//             l = 16 q + c supplies rows 8 q .. 8 q + 7 of column c of a 32-row
//             block as the A operand, the B operand is the W part tile of that
//             row block.  T leaves as three BF16 parts in the B-operand order of
//             the second kernel (contraction over columns).
//   k_mc_xt   partial X T for 256 rows and one column range.  A 256 x 32 tile
//             of X is read column by column (coalesced) and kept column by
//             column in LDS; each lane gathers 8 consecutive columns of its row
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
constexpr int XT_MT = 2;             // 16-row tiles per wave in k_mc_xt
constexpr int RB = NW * 16 * XT_MT;  // rows per k_mc_xt workgroup
constexpr int XTW_COLS = NW * 16;   // columns per k_mc_xtw workgroup

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

// One 16-byte chunk (4 FP32 or 8 BF16 values) of a column from row r, as
// load8 does it: VEC (d % 8 == 0) moves a chunk past d back to the last whole
// chunk, the scalar form clamps each row to d - 1.
template <typename TX, bool VEC>
__device__ __forceinline__ u32x4 load_chunk(const TX* __restrict__ col, int64_t r, int64_t d) {
  constexpr int E = 16 / (int)sizeof(TX);
  if constexpr (VEC) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const u32x4*>(col + (r + E <= d ? r : d - E)));
  } else if constexpr (sizeof(TX) == 2) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      w[h] = (uint32_t)col[imin(r + 2 * h, d - 1)] | ((uint32_t)col[imin(r + 2 * h + 1, d - 1)] << 16);
    return u32x4{w[0], w[1], w[2], w[3]};
  } else {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = __float_as_uint(col[imin(r + i, d - 1)]);
    return u32x4{w[0], w[1], w[2], w[3]};
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

// T = X^T W for 128 columns per workgroup, all rows, in stages of 64 rows.
// A stage's 128 x 64 tile of X is fetched column by column (the threads of
// one column read its rows as one contiguous run of 128 or 256 bytes), kept in
// registers two stages ahead and written to the other LDS buffer; the W part
// tiles of the stage's two row blocks travel the same way.  Wave w multiplies
// column tile w over every row block (lane 16 q + c reads rows 8 q .. 8 q + 7
// of column c of a 32-row block from LDS as the A operand).  Each W part tile
// staged in LDS thus serves 128 columns of X, which keeps the tiles' share of
// the on-chip traffic below X's own.  One barrier per stage; every load reads
// an in-bounds address outside any branch.
template <typename TX, int NTW, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_mc_xtw(const TX* __restrict__ X, int64_t ld,
                                                    int64_t d, int64_t n,
                                                    const uint16_t* __restrict__ Wp,
                                                    int64_t wstride, uint16_t* __restrict__ Tp,
                                                    int64_t tstride, int64_t tcols) {
  using XT = XTraits<TX>;
  constexpr int NPX = XT::NPX, NV = XT::NV;
  constexpr int CB = XTW_COLS;                           // columns per workgroup
  constexpr int KPS = 2;                                 // 32-row blocks per stage
  static_assert(CB == 16 * NW, "one 16-column tile per wave");
  constexpr int RS = 32 * KPS;                           // rows per stage
  constexpr int EPC = 16 / (int)sizeof(TX);              // elements per 16-byte chunk
  constexpr int CPC = RS / EPC;                          // chunks per column per stage
  constexpr int XW = CB * CPC / (NW * 64);               // X chunks per thread per stage
  constexpr int LDX = RS + EPC;                          // LDS column pitch (elements)
  constexpr int TILES = KPS * NPART * NTW;               // W part tiles per stage
  constexpr int WW = (TILES * 64 + NW * 64 - 1) / (NW * 64);
  static_assert(CB * CPC % (NW * 64) == 0, "whole chunks per thread");
  __shared__ __align__(16) TX xs[2][CB * LDX];
  __shared__ u32x4 wsh[2][WW * NW * 64];                 // words past TILES * 64 are never read
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = NTW;
  const int mt = wave;                                   // column tile
  const int64_t c0 = (int64_t)blockIdx.x * CB;
  const int64_t nst = (d + RS - 1) / RS;
  struct Stage {
    u32x4 x[XW];
    u32x4 w[WW];
  };
  auto load = [&](Stage& S, int64_t st) {
    st = imin(st, nst - 1);
#pragma unroll
    for (int j = 0; j < XW; ++j) {
      const int e = t + j * NW * 64, cc = e / CPC, ch = e % CPC;
      const TX* __restrict__ col = X + imin(c0 + cc, n - 1) * ld;
      const int64_t r = st * RS + (int64_t)ch * EPC;
      S.x[j] = load_chunk<TX, VEC>(col, r, d);
    }
#pragma unroll
    for (int j = 0; j < WW; ++j) {
      int e = t + j * NW * 64;
      e = e < TILES * 64 ? e : TILES * 64 - 1;
      const int tile = e / 64, kb = tile / (NPART * NTW), g = (tile / NTW) % NPART, u = tile % NTW;
      // the W parts hold zero rows up to a multiple of 128, so a stage past d
      // meets zeros
      const int64_t kbg = st * KPS + kb;
      S.w[j] = *reinterpret_cast<const u32x4*>(Wp + g * wstride + ((kbg * NS + u) * 64 + e % 64) * 8);
    }
  };
  auto stage_lds = [&](const Stage& S, int buf) {
#pragma unroll
    for (int j = 0; j < XW; ++j) {
      const int e = t + j * NW * 64, cc = e / CPC, ch = e % CPC;
      *reinterpret_cast<u32x4*>(&xs[buf][cc * LDX + ch * EPC]) = S.x[j];
    }
#pragma unroll
    for (int j = 0; j < WW; ++j) wsh[buf][t + j * NW * 64] = S.w[j];
  };
  f32x4 acc[NTW];
  double accd[NTW][4];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) accd[u][v] = 0.0;
  }
  int since = 0;   // row blocks accumulated in FP32 since the last flush
  auto flush = [&]() {
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[u][v] += (double)acc[u][v];
      acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kb = 0; kb < KPS; ++kb) {
      const TX* xa = &xs[buf][(mt * 16 + li) * LDX + kb * 32 + 8 * q];
      u32x4 av[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) av[i] = reinterpret_cast<const u32x4*>(xa)[i];
      bf16x8 xp[NPX];
      a_parts<TX>(av, xp);
#pragma unroll
      for (int g = 0; g < NPART; ++g)
#pragma unroll
        for (int u = 0; u < NTW; ++u) {
          const bf16x8 wf =
              __builtin_bit_cast(bf16x8, wsh[buf][((kb * NPART + g) * NTW + u) * 64 + l]);
#pragma unroll
          for (int h = 0; h < NPX; ++h)
            if (h + g < NPART) acc[u] = mfma(xp[h], wf, acc[u]);
        }
    }
  };
  // stage st + 1 goes to LDS (its loads were issued two stages earlier) and its
  // registers are refilled with stage st + 3 while stage st is multiplied
  auto step = [&](int64_t st, Stage& nxt) {
    stage_lds(nxt, (int)((st + 1) & 1));
    load(nxt, st + 3);
    compute((int)(st & 1));
    since += KPS;
    if (since >= FLUSH) {
      flush();
      since = 0;
    }
    __syncthreads();
  };
  {
    Stage A, B;
    load(A, 0);
    load(B, 1);
    stage_lds(A, 0);
    load(A, 2);
    __syncthreads();
    int64_t st = 0;
    for (; st + 2 <= nst; st += 2) {
      step(st, B);
      step(st + 1, A);
    }
    if (st < nst) step(st, B);
  }
  flush();
  // wave mt holds T[c0 + 16 mt + 4 q + v][16 u + c];
  // lanes with even q take their partner's four rows and store eight
  // consecutive columns of T (one 16-byte word per part), zero past n
  __bf16* tout = reinterpret_cast<__bf16*>(Tp);
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    double v8[8];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      v8[v] = accd[u][v];
      v8[4 + v] = __shfl_down(accd[u][v], 16);
    }
    const int64_t ca = c0 + 16 * mt + 4 * q;
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
}

// Partial sums of X T over the columns of split s for rows r0 .. r0 + RB - 1;
// workgroup -> (split, row block) keeps every row block of a split on one XCD
// so the split's T tiles are fetched into one L2, and a row block of 256 rows
// (two 16-row tiles per wave) halves how often each T tile is fetched and read
// from LDS against 128 rows.  Each thread fetches one column's 8-row chunks of
// the next-but-one 32-column block and its share of the T part tiles; a block
// is staged in the other LDS buffer while the current one is multiplied, one
// barrier per block.
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
  // X tile in LDS column by column, pitch CP elements: a thread's 8 rows of one
  // column go in as 8-byte stores, and the 64 lanes reading column 8 q + i of
  // rows 16 t + c of tile t meet 64 distinct banks (CP = RB + 2 = 258 words, 2 mod 64;
  // BF16: 130 words, also 2 mod 64, two lanes sharing each word)
  constexpr int CP = sizeof(TX) == 4 ? RB + 2 : RB + 4;
  __shared__ __align__(16) TX xs[2][32 * CP];
  __shared__ u32x4 ts[2][TPT * NW * 64];   // words past TT * 64 are never read
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = NTW;
  const int id = blockIdx.x, loc = id / 8;
  const int64_t s = (int64_t)(loc / nrb) * 8 + id % 8;
  const int64_t r0 = (int64_t)(loc % nrb) * RB;
  const int64_t kb0 = s * kper / 32;
  const int64_t kb1 = imin((s + 1) * kper, (n + 31) / 32 * 32) / 32;
  // loader: column cc of the block, rows rr + 128 h .. + 7 of the row block (h < XT_MT)
  const int cc = t / 16, rr = (t % 16) * 8;
  struct Stage {
    u32x4 x[XT_MT][NV];
    u32x4 tw[TPT];
  };
  auto load = [&](Stage& S, int64_t kb) {
    kb = imin(kb, kb1 - 1);
    const int64_t col = imin(kb * 32 + cc, n - 1);
#pragma unroll
    for (int h = 0; h < XT_MT; ++h) load8<TX, VEC>(X + col * ld, r0 + rr + 128 * h, d, S.x[h]);
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
    for (int h = 0; h < XT_MT; ++h) {
      uint32_t* dst = reinterpret_cast<uint32_t*>(&xs[buf][cc * CP + rr + 128 * h]);
      if constexpr (sizeof(TX) == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          reinterpret_cast<uint2*>(dst)[i] =
              make_uint2(S.x[h][i / 2][2 * (i % 2)], S.x[h][i / 2][2 * (i % 2) + 1]);
      } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          reinterpret_cast<uint2*>(dst)[i] = make_uint2(S.x[h][0][2 * i], S.x[h][0][2 * i + 1]);
      }
    }
#pragma unroll
    for (int i = 0; i < TPT; ++i) ts[buf][t + i * NW * 64] = S.tw[i];
  };
  f32x4 acc[XT_MT][NTW];
  double accd[XT_MT][NTW][4];
#pragma unroll
  for (int mt = 0; mt < XT_MT; ++mt)
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
      acc[mt][u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[mt][u][v] = 0.0;
    }
  // wave w owns row tiles XT_MT w .. XT_MT w + XT_MT - 1; each T part tile read
  // from LDS serves all of them
  auto compute = [&](int buf) {
    bf16x8 xp[XT_MT][NPX];
#pragma unroll
    for (int mt = 0; mt < XT_MT; ++mt) {
      // column 8 q of the block, row 16 (XT_MT w + mt) + c
      const int arow = 8 * q * CP + (wave * XT_MT + mt) * 16 + li;
      u32x4 av[NV];
      if constexpr (sizeof(TX) == 4) {
        const uint32_t* xw = reinterpret_cast<const uint32_t*>(xs[buf]) + arow;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          av[0][i] = xw[i * CP];
          av[1][i] = xw[(4 + i) * CP];
        }
      } else {
        const uint16_t* xh = reinterpret_cast<const uint16_t*>(xs[buf]) + arow;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          av[0][i] = (uint32_t)xh[2 * i * CP] | ((uint32_t)xh[(2 * i + 1) * CP] << 16);
      }
      a_parts<TX>(av, xp[mt]);
    }
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int g = 0; g < NPART; ++g) {
        const bf16x8 tb = __builtin_bit_cast(bf16x8, ts[buf][(g * NTW + u) * 64 + l]);
#pragma unroll
        for (int mt = 0; mt < XT_MT; ++mt)
#pragma unroll
          for (int h = 0; h < NPX; ++h)
            if (h + g < NPART) acc[mt][u] = mfma(xp[mt][h], tb, acc[mt][u]);
      }
  };
  auto flush = [&]() {
#pragma unroll
    for (int mt = 0; mt < XT_MT; ++mt)
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[mt][u][v] += (double)acc[mt][u][v];
        acc[mt][u] = f32x4{0.f, 0.f, 0.f, 0.f};
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
  for (int mt = 0; mt < XT_MT; ++mt)
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + (wave * XT_MT + mt) * 16 + 4 * q + v;
        out[r * (NTW * 16) + 16 * u + li] = (float)accd[mt][u][v];
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
  // about 256 workgroups, one per compute unit (fewer, longer column runs
  // stream better, and the partials to reduce shrink with the split count);
  // a multiple of 8 splits for the XCD mapping
  int64_t ns = round_up(std::max<int64_t>(8, (256 + sp.nrb - 1) / sp.nrb), 8);
  // and at least 256 columns per split, so a short X does not leave most of the
  // pass to the reduce of many one-block partials
  ns = std::min<int64_t>(ns, round_up(std::max<int64_t>(1, (n + 255) / 256), 8));
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
  z.wp_elems = (int64_t)NPART * round_up(d, 128) * PC;   // zero rows up to a stage multiple
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
  const int64_t wstride = round_up(X.d, 128) * PC, tstride = round_up(X.n, 32) * PC;
  if (sp.nsplit != mb.nsplit || wstride != mb.wstride || tstride != mb.tstride)
    return hipErrorInvalidValue;
  const int64_t pstride = (int64_t)sp.nrb * RB * PC;
  const int64_t wrows = round_up(X.d, 128);
  k_mc_split_w<<<(unsigned)((wrows * PC + 255) / 256), 256, 0, st>>>(W, X.d, p, PC, wrows, mb.Wp,
                                                                     wstride);
  const int64_t tcols = round_up(X.n, 32);
  const bool vec = X.d % 8 == 0 && X.d >= 8;
  const dim3 g1((unsigned)((X.n + XTW_COLS - 1) / XTW_COLS));
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
