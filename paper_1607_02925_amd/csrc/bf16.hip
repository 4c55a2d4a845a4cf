// BF16 matrix-core inner steps for dense BF16 X (gfx950 v_mfma_f32_16x16x32_bf16).
//
// The instruction multiplies a 16 x 32 A by a 32 x 16 B: lane l supplies row
// l % 16 of A and column l % 16 of B over k = 8 (l / 16) + t, t < 8 (the same k
// for both operands), and receives D[4 (l / 16) + v][l % 16] in accumulator v.
// Eight consecutive k of one lane are eight consecutive rows (or samples) in
// memory, so X columns and the split operands are fetched 16 bytes per lane.
#include "bf16.h"

#include <hip/hip_ext.h>

namespace lr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KST = 8192;   // largest minibatch; its indices are staged in LDS

__device__ __forceinline__ f32x4 mfma_bf16(const uint4& a, const uint4& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Round-to-nearest-even BF16 bit pattern of a finite float.
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void split2(double x, uint16_t* hi, uint16_t* lo) {
  const uint16_t h = bf16_rne((float)x);
  *hi = h;
  *lo = bf16_rne((float)(x - (double)__uint_as_float((uint32_t)h << 16)));
}

// The split operands (Dh/Dlo of the step difference, Ch/Cl of C) are kept in
// the matrix-core B-operand order: for each block of 32 k (rows of d, or
// samples) and each 16-column slice a contiguous tile of 512 BF16 values in
// which lane l = 16 q + c holds k = 8 q .. 8 q + 7 of column c.  A wave reads
// a tile as one contiguous 1 KB load; rows past d (or samples past b) and
// columns past p stay zero.
__device__ __forceinline__ int64_t bt_off(int64_t k, int j, int NS) {
  const int w = (int)(k & 31);
  return (((k >> 5) * NS + (j >> 4)) * 64 + (w >> 3) * 16 + (j & 15)) * 8 + (w & 7);
}

__device__ __forceinline__ uint4 tile_b(const uint16_t* __restrict__ base, int64_t kb, int u,
                                        int NS, int l) {
  return *reinterpret_cast<const uint4*>(base + ((kb * NS + u) * 64 + l) * 8);
}

// Eight consecutive BF16 values of one column from row r, all rows < d.
template <bool VEC>
__device__ __forceinline__ uint4 load8full(const uint16_t* __restrict__ col, int64_t r) {
  if constexpr (VEC) return *reinterpret_cast<const uint4*>(col + r);
  uint32_t w[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) w[h] = (uint32_t)col[r + 2 * h] | ((uint32_t)col[r + 2 * h + 1] << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// The same with rows >= d read as zero (addresses clamped to row d - 1).
__device__ __forceinline__ uint4 load8tail(const uint16_t* __restrict__ col, int64_t r, int64_t d) {
  uint32_t w[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int64_t ra = r + 2 * h, rb = ra + 1;
    const uint32_t va = col[min(ra, d - 1)], vb = col[min(rb, d - 1)];
    w[h] = (ra < d ? va : 0u) | ((rb < d ? vb : 0u) << 16);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// C = diag(scale) X_B^T (Dh + Dlo) for 16 samples x NTW 16-column slices; the
// NW waves split the rows in 32-row blocks.  Two register stages of G blocks:
// the next stage's loads are issued before the current stage's matrix-core
// work.  Every load reads an in-bounds address: samples past b read column
// idx[0] (their rows of C are not stored), a stage's blocks past the wave's
// range re-read its last block and skip their matrix-core work on a
// wave-uniform branch, and the partial last block of rows is done on its own
// with clamped, zeroed X loads (the split tiles hold zeros past d).
template <int NW, int NTW, int G, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_sdot_bf16(
    const uint16_t* __restrict__ X, int64_t ld, int64_t d, int64_t b,
    const int32_t* __restrict__ idx, const double* __restrict__ scale,
    const uint16_t* __restrict__ Dh, const uint16_t* __restrict__ Dlo,
    uint16_t* __restrict__ Ch, uint16_t* __restrict__ Cl, int PC) {
  __shared__ double slots[NW * NTW * 256];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = PC / 16;
  const int64_t s0 = (int64_t)blockIdx.x * 16;
  const int64_t s = s0 + li;
  const uint16_t* __restrict__ xcol = X + (int64_t)idx[s < b ? s : 0] * ld;
  // the epilogue's weight, loaded now so that its latency hides under the loop
  // (thread t writes sample row i = (t / 16) % 16 of every slice)
  static_assert((NW * 64) % 256 == 0, "a thread keeps its sample row across slices");
  const int64_t sw = s0 + (t / 16) % 16;
  const double wsc = scale[sw < b ? sw : 0];
  f32x4 ah[NTW], al[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) ah[u] = al[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nkb = (d + 31) / 32, nfull = d / 32;
  const int64_t kpw = (nkb + NW - 1) / NW;
  const int64_t k0 = wave * kpw, k1 = min(nkb, k0 + kpw);
  const int64_t kend = min(k1, nfull);
  struct Stage {
    uint4 xa[G], bh[G][NTW], bl[G][NTW];
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t kb = min(g + i, kend - 1);
      S.xa[i] = load8full<VEC>(xcol, kb * 32 + 8 * q);
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        S.bh[i][u] = tile_b(Dh, kb, u, NS, l);
        S.bl[i][u] = tile_b(Dlo, kb, u, NS, l);
      }
    }
  };
  auto compute = [&](const Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (g + i >= kend) break;
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        ah[u] = mfma_bf16(S.xa[i], S.bh[i][u], ah[u]);
        al[u] = mfma_bf16(S.xa[i], S.bl[i][u], al[u]);
      }
    }
  };
  if (k0 < kend) {
    Stage A, B;
    load(A, k0);
    for (int64_t g = k0; g < kend; g += 2 * G) {
      load(B, g + G);
      __builtin_amdgcn_sched_barrier(0);
      compute(A, g);
      load(A, g + 2 * G);
      __builtin_amdgcn_sched_barrier(0);
      compute(B, g + G);
    }
  }
  if (nfull < nkb && k0 <= nfull && nfull < k1) {   // the partial last block of rows
    const uint4 xa = load8tail(xcol, nfull * 32 + 8 * q, d);
#pragma unroll
    for (int u = 0; u < NTW; ++u) {
      ah[u] = mfma_bf16(xa, tile_b(Dh, nfull, u, NS, l), ah[u]);
      al[u] = mfma_bf16(xa, tile_b(Dlo, nfull, u, NS, l), al[u]);
    }
  }
  double* mine = slots + wave * (NTW * 256);
#pragma unroll
  for (int u = 0; u < NTW; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      mine[u * 256 + (4 * q + v) * 16 + li] = (double)ah[u][v] + (double)al[u][v];
  __syncthreads();
  for (int e = t; e < NTW * 256; e += NW * 64) {
    double sum = slots[e];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += slots[w * (NTW * 256) + e];
    const int u = e / 256, i = (e / 16) % 16, jj = e % 16;
    const int64_t ss = s0 + i;
    if (ss < b) {
      const int64_t o = bt_off(ss, u * 16 + jj, NS);
      split2(wsc * sum, &Ch[o], &Cl[o]);
    }
  }
}

// v from lane l ^ 2 of the same quad of lanes (DPP quad_perm [2, 3, 0, 1]).
__device__ __forceinline__ uint32_t quad_xor2(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
}

// Orders a wave's LDS accesses around it (a wave's own LDS operations complete
// in issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// U = X_B (Ch + Cl)^T for 16 rows x NTW slices; Dl <- Dl - eta (G + lam Dl - U)
// for r < d, j < p, and the new Dl is split into Dh/Dlo.  The NW waves split
// the samples in 32-sample blocks; the indices are staged in LDS, padded to a
// multiple of 32 with a valid column (the split C tiles hold zeros past b), so
// every block is whole.  A block comes in with one 16-byte load per lane: lane
// l takes rows 8 (l % 2) .. + 7 of the row tile from sample l / 2 (VEC moves a
// piece past d back to rows d - 8 .. d - 1, the scalar form reads rows past d
// as zero; rows past d are not stored).  Lanes l and l ^ 2 (samples 2 m and
// 2 m + 1) swap half their rows by DPP so that each holds four words (row,
// samples 2 m, 2 m + 1), which the wave writes into its own LDS tile (two,
// alternating; rows of 16 words at a pitch of 20, so the 64 lanes' writes meet
// 64 banks) and reads back in the matrix-core operand order: row l % 16,
// samples 8 (l / 16) .. + 7 as one 16-byte read.  Two register stages, taken
// in whole pairs without a branch so that the next stage's loads stay ahead
// of the current stage's work.  The grid (a multiple of 8 tiles) is remapped
// so that each XCD owns a contiguous run of row tiles and the pieces of a
// gathered column's cache line meet in one L2.
template <int NW, int NTW, int G, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_supd_bf16(
    const uint16_t* __restrict__ X, int64_t ld, int64_t d, int64_t b,
    const int32_t* __restrict__ idx, const uint16_t* __restrict__ Ch,
    const uint16_t* __restrict__ Cl, int PC, int p, const double* __restrict__ Gr,
    double* __restrict__ Dl, uint16_t* __restrict__ Dh, uint16_t* __restrict__ Dlo,
    double lam, double eta) {
  constexpr int EPT = (NTW * 256 + NW * 64 - 1) / (NW * 64);
  constexpr int XTP = 20;   // words per row of a transpose tile
  __shared__ double slots[NW * NTW * 256];
  __shared__ int sidx[KST];
  __shared__ __align__(16) uint32_t xtr[NW][2][16 * XTP];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int NS = PC / 16;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int64_t r0 = tile * 16;
  if (r0 >= d) return;
  // the epilogue's operands are fetched now, so their latency overlaps the loop
  double e_dl[EPT], e_g[EPT];
  int64_t eo[EPT], er[EPT];
  int ej[EPT];
  bool ev[EPT];
#pragma unroll
  for (int a = 0; a < EPT; ++a) {
    const int e = t + a * NW * 64;
    er[a] = r0 + (e % 256) / 16;
    ej[a] = e / 256 * 16 + e % 16;
    ev[a] = e < NTW * 256 && er[a] < d && ej[a] < p;
    eo[a] = ev[a] ? (int64_t)ej[a] * d + er[a] : 0;
    e_dl[a] = ev[a] ? Dl[eo[a]] : 0.0;
    e_g[a] = ev[a] ? Gr[eo[a]] : 0.0;
  }
  const int64_t bpad = (b + 31) / 32 * 32;
  for (int64_t e = t; e < bpad; e += NW * 64) sidx[e] = idx[e < b ? e : 0];
  __syncthreads();
  const int lj = l >> 1, lh = 8 * (l & 1);   // this lane's sample and first row in a block
  const int64_t rr = r0 + lh;
  const int64_t rl = VEC && rr + 8 > d ? d - 8 : rr;
  // after the exchange: rows wr0 .. wr0 + 3 of the sample pair wm
  const bool even = (l & 2) == 0;
  const int wr0 = lh + (even ? 0 : 4), wm = lj >> 1;
  f32x4 ah[NTW], al[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) ah[u] = al[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nkb = bpad / 32;
  const int64_t kpw = (nkb + NW - 1) / NW;
  const int64_t k0 = wave * kpw, k1 = min(nkb, k0 + kpw);
  struct Stage {
    uint4 xa[G], ch[G][NTW], cl[G][NTW];
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t kb = min(g + i, k1 - 1);
      const uint16_t* __restrict__ col = X + (int64_t)sidx[kb * 32 + lj] * ld;
      S.xa[i] = VEC ? load8full<true>(col, rl) : load8tail(col, rr, d);
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        S.ch[i][u] = tile_b(Ch, kb, u, NS, l);
        S.cl[i][u] = tile_b(Cl, kb, u, NS, l);
      }
    }
  };
  auto compute = [&](const Stage& S, int64_t g, bool checked) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (checked && g + i >= k1) break;
      // words (row, samples 2 wm and 2 wm + 1): the even lane of a pair keeps
      // its first four rows and takes its partner's, the odd lane the last four
      const uint4 w = S.xa[i];
      const uint32_t r0w = quad_xor2(even ? w.z : w.x), r1w = quad_xor2(even ? w.w : w.y);
      const uint32_t a0 = even ? w.x : r0w, a1 = even ? w.y : r1w;   // sample 2 wm
      const uint32_t b0 = even ? r0w : w.z, b1 = even ? r1w : w.w;   // sample 2 wm + 1
      uint32_t* __restrict__ wt = xtr[wave][(g + i) & 1];
      wt[(wr0 + 0) * XTP + wm] = (a0 & 0xFFFFu) | (b0 << 16);
      wt[(wr0 + 1) * XTP + wm] = (a0 >> 16) | (b0 & 0xFFFF0000u);
      wt[(wr0 + 2) * XTP + wm] = (a1 & 0xFFFFu) | (b1 << 16);
      wt[(wr0 + 3) * XTP + wm] = (a1 >> 16) | (b1 & 0xFFFF0000u);
      wave_sync();
      const uint4 xa = *reinterpret_cast<const uint4*>(wt + li * XTP + 4 * q);
      wave_sync();
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        ah[u] = mfma_bf16(xa, S.ch[i][u], ah[u]);
        al[u] = mfma_bf16(xa, S.cl[i][u], al[u]);
      }
    }
  };
  if (k0 < k1) {
    Stage A, B;
    load(A, k0);
    int64_t g = k0;
    for (; g + 2 * G <= k1; g += 2 * G) {
      load(B, g + G);
      __builtin_amdgcn_sched_barrier(0);
      compute(A, g, false);
      load(A, g + 2 * G);
      __builtin_amdgcn_sched_barrier(0);
      compute(B, g + G, false);
    }
    if (g < k1) {
      compute(A, g, true);
      if (g + G < k1) {
        load(B, g + G);
        compute(B, g + G, true);
      }
    }
  }
  double* mine = slots + wave * (NTW * 256);
#pragma unroll
  for (int u = 0; u < NTW; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      mine[u * 256 + (4 * q + v) * 16 + li] = (double)ah[u][v] + (double)al[u][v];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < EPT; ++a) {
    const int e = t + a * NW * 64;
    if (!ev[a]) continue;
    double U = slots[e];
#pragma unroll
    for (int w = 1; w < NW; ++w) U += slots[w * (NTW * 256) + e];
    const double x = e_dl[a] - eta * (e_g[a] + lam * e_dl[a] - U);
    Dl[eo[a]] = x;
    const int64_t o = bt_off(er[a], ej[a], NS);
    split2(x, &Dh[o], &Dlo[o]);
  }
}

}  // namespace

int64_t pad_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

template <typename K, typename... A>
static void launch_bf(K kernel, dim3 grid, dim3 block, hipStream_t st, const Probe& pr,
                      A... args) {
  if (pr.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pr.start, pr.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

#define BF_DISPATCH_NTW(nt, NTW, ...) \
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

hipError_t step_dot_bf16(const XView& X, int p, int64_t b, const int32_t* idx,
                         const double* scale, const uint16_t* Dh, const uint16_t* Dlo,
                         int64_t ldD, uint16_t* Ch, uint16_t* Cl, int64_t ldC, int PC,
                         hipStream_t st, const Probe& pr) {
  if (X.dt != 2 || PC % 16 || PC > 64 || p > PC || ldD % 32 || ldD < X.d || ldC % 32 ||
      ldC < pad_to(b, 32) || (uintptr_t)Dh % 16 || (uintptr_t)Dlo % 16)
    return hipErrorInvalidValue;
  const bool vec = X.ld % 8 == 0 && (uintptr_t)X.v % 16 == 0;
  const dim3 grid((unsigned)((b + 15) / 16), 1);
  BF_DISPATCH_NTW(PC / 16, NTW, {
    constexpr int GB = NTW <= 2 ? 2 : 1;
    if (vec)
      launch_bf(k_sdot_bf16<8, NTW, GB, true>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, scale, Dh, Dlo, Ch, Cl, PC);
    else
      launch_bf(k_sdot_bf16<8, NTW, GB, false>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, scale, Dh, Dlo, Ch, Cl, PC);
  });
  return hipGetLastError();
}

hipError_t step_update_bf16(const XView& X, int p, int64_t b, const int32_t* idx,
                            const uint16_t* Ch, const uint16_t* Cl, int64_t ldC, int PC,
                            const double* G, double* Dl, uint16_t* Dh, uint16_t* Dlo,
                            int64_t ldD, double lam, double eta, hipStream_t st,
                            const Probe& pr) {
  if (X.dt != 2 || b > KST || PC % 16 || PC > 64 || p > PC || ldD % 32 || ldD < X.d ||
      ldC % 32 || ldC < pad_to(b, 32) || (uintptr_t)Ch % 16 || (uintptr_t)Cl % 16)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((X.d + 15) / 16 + 7) / 8 * 8), 1);
  // 16-byte pieces of 8 rows: aligned columns, d a multiple of 8
  const bool vec = X.ld % 8 == 0 && X.d % 8 == 0 && (uintptr_t)X.v % 16 == 0;
  BF_DISPATCH_NTW(PC / 16, NTW, {
    constexpr int GB = NTW <= 2 ? 2 : 1;
    if (vec)
      launch_bf(k_supd_bf16<8, NTW, GB, true>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, Ch, Cl, PC, p, G, Dl, Dh, Dlo, lam, eta);
    else
      launch_bf(k_supd_bf16<8, NTW, GB, false>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, Ch, Cl, PC, p, G, Dl, Dh, Dlo, lam, eta);
  });
  return hipGetLastError();
}

}  // namespace lr
