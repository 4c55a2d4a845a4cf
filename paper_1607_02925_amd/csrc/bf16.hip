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

// Eight consecutive BF16 values of one column from row r (zeros beyond d).
template <bool VEC>
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ col, int64_t r, int64_t d) {
  if (VEC && r + 7 < d) return *reinterpret_cast<const uint4*>(col + r);
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t a = r + 2 * q < d ? (uint32_t)col[r + 2 * q] : 0u;
    const uint32_t b = r + 2 * q + 1 < d ? (uint32_t)col[r + 2 * q + 1] : 0u;
    w[q] = a | (b << 16);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// C = diag(scale) X_B^T (Dh + Dlo) for 16 samples x NTW 16-column slices; the
// NW waves split the rows in 32-row blocks and fetch G blocks ahead.
template <int NW, int NTW, int G, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_sdot_bf16(
    const uint16_t* __restrict__ X, int64_t ld, int64_t d, int64_t b,
    const int32_t* __restrict__ idx, const double* __restrict__ scale,
    const uint16_t* __restrict__ Dh, const uint16_t* __restrict__ Dlo, int64_t ldD,
    uint16_t* __restrict__ Ch, uint16_t* __restrict__ Cl, int64_t ldC, int PC) {
  __shared__ double slots[NW * NTW * 256];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int64_t s0 = (int64_t)blockIdx.x * 16;
  const int nt0 = blockIdx.y * NTW;
  const int64_t s = s0 + li;
  const bool sval = s < b;
  const uint16_t* xcol = X + (sval ? (int64_t)idx[s] : 0) * ld;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  f32x4 ah[NTW], al[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) ah[u] = al[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nkb = (d + 31) / 32;
  const int64_t kpw = (nkb + NW - 1) / NW;
  const int64_t k0 = wave * kpw, k1 = min(nkb, k0 + kpw);
  for (int64_t g0 = k0; g0 < k1; g0 += G) {
    uint4 xa[G], bh[G][NTW], bl[G][NTW];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t r = (g0 + i) * 32 + 8 * q;
      const bool kv = g0 + i < k1;
      xa[i] = (kv && sval) ? load8<VEC>(xcol, r, d) : z4;
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const bool jv = kv && (nt0 + u) * 16 < PC;
        const int64_t o = (int64_t)((nt0 + u) * 16 + li) * ldD + r;
        bh[i][u] = jv ? *reinterpret_cast<const uint4*>(Dh + o) : z4;
        bl[i][u] = jv ? *reinterpret_cast<const uint4*>(Dlo + o) : z4;
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i)
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        ah[u] = mfma_bf16(xa[i], bh[i][u], ah[u]);
        al[u] = mfma_bf16(xa[i], bl[i][u], al[u]);
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
    if (ss < b && (nt0 + u) * 16 < PC) {
      const int64_t o = (int64_t)((nt0 + u) * 16 + jj) * ldC + ss;
      split2(scale[ss] * sum, &Ch[o], &Cl[o]);
    }
  }
}

// U = X_B (Ch + Cl)^T for 16 rows x NTW slices; Dl <- Dl - eta (G + lam Dl - U)
// for r < d, j < p, and the new Dl is split into Dh/Dlo.  The NW waves split
// the samples in 32-sample blocks (indices staged in LDS).
template <int NW, int NTW, int G>
__global__ __launch_bounds__(NW * 64) void k_supd_bf16(
    const uint16_t* __restrict__ X, int64_t ld, int64_t d, int64_t b,
    const int32_t* __restrict__ idx, const uint16_t* __restrict__ Ch,
    const uint16_t* __restrict__ Cl, int64_t ldC, int PC, int p, const double* __restrict__ Gr,
    double* __restrict__ Dl, uint16_t* __restrict__ Dh, uint16_t* __restrict__ Dlo,
    int64_t ldD, double lam, double eta) {
  constexpr int EPT = (NTW * 256 + NW * 64 - 1) / (NW * 64);
  __shared__ double slots[NW * NTW * 256];
  __shared__ int sidx[KST];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, li = l % 16, q = l / 16;
  const int64_t r0 = (int64_t)blockIdx.x * 16;
  const int nt0 = blockIdx.y * NTW;
  // the epilogue's operands are fetched now, so their latency overlaps the loop
  double e_dl[EPT], e_g[EPT];
  int64_t eo[EPT], er[EPT];
  int ej[EPT];
  bool ev[EPT];
#pragma unroll
  for (int a = 0; a < EPT; ++a) {
    const int e = t + a * NW * 64;
    er[a] = r0 + (e % 256) / 16;
    ej[a] = (nt0 + e / 256) * 16 + e % 16;
    ev[a] = e < NTW * 256 && er[a] < d && ej[a] < p;
    eo[a] = ev[a] ? (int64_t)ej[a] * d + er[a] : 0;
    e_dl[a] = ev[a] ? Dl[eo[a]] : 0.0;
    e_g[a] = ev[a] ? Gr[eo[a]] : 0.0;
  }
  for (int64_t e = t; e < b; e += NW * 64) sidx[e] = idx[e];
  __syncthreads();
  const int64_t row = r0 + li;
  const bool rval = row < d;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  f32x4 ah[NTW], al[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) ah[u] = al[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nkb = (b + 31) / 32;
  const int64_t kpw = (nkb + NW - 1) / NW;
  const int64_t k0 = wave * kpw, k1 = min(nkb, k0 + kpw);
  for (int64_t g0 = k0; g0 < k1; g0 += G) {
    uint4 xa[G], ch[G][NTW], cl[G][NTW];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t sb = (g0 + i) * 32 + 8 * q;
      const bool kv = g0 + i < k1;
      uint32_t w[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int64_t sa = sb + 2 * h, sc = sa + 1;
        const uint32_t a = (kv && rval && sa < b) ? (uint32_t)X[(int64_t)sidx[sa] * ld + row] : 0u;
        const uint32_t c = (kv && rval && sc < b) ? (uint32_t)X[(int64_t)sidx[sc] * ld + row] : 0u;
        w[h] = a | (c << 16);
      }
      xa[i] = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const bool jv = kv && (nt0 + u) * 16 < PC;
        const int64_t o = (int64_t)((nt0 + u) * 16 + li) * ldC + sb;
        ch[i][u] = jv ? *reinterpret_cast<const uint4*>(Ch + o) : z4;
        cl[i][u] = jv ? *reinterpret_cast<const uint4*>(Cl + o) : z4;
      }
    }
#pragma unroll
    for (int i = 0; i < G; ++i)
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        ah[u] = mfma_bf16(xa[i], ch[i][u], ah[u]);
        al[u] = mfma_bf16(xa[i], cl[i][u], al[u]);
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
    const int64_t o = (int64_t)ej[a] * ldD + er[a];
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
      ldC < pad_to(b, 32))
    return hipErrorInvalidValue;
  const bool vec = X.ld % 8 == 0 && (uintptr_t)X.v % 16 == 0;
  const dim3 grid((unsigned)((b + 15) / 16), 1);
  BF_DISPATCH_NTW(PC / 16, NTW, {
    constexpr int GB = NTW <= 2 ? 4 : 2;
    if (vec)
      launch_bf(k_sdot_bf16<8, NTW, GB, true>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, scale, Dh, Dlo, ldD, Ch, Cl, ldC, PC);
    else
      launch_bf(k_sdot_bf16<8, NTW, GB, false>, grid, dim3(512), st, pr, (const uint16_t*)X.v,
                X.ld, X.d, b, idx, scale, Dh, Dlo, ldD, Ch, Cl, ldC, PC);
  });
  return hipGetLastError();
}

hipError_t step_update_bf16(const XView& X, int p, int64_t b, const int32_t* idx,
                            const uint16_t* Ch, const uint16_t* Cl, int64_t ldC, int PC,
                            const double* G, double* Dl, uint16_t* Dh, uint16_t* Dlo,
                            int64_t ldD, double lam, double eta, hipStream_t st,
                            const Probe& pr) {
  if (X.dt != 2 || b > KST || PC % 16 || PC > 64 || p > PC || ldD % 32 || ldD < X.d ||
      ldC % 32 || ldC < pad_to(b, 32))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((X.d + 15) / 16), 1);
  BF_DISPATCH_NTW(PC / 16, NTW, {
    constexpr int GB = NTW <= 2 ? 4 : 2;
    launch_bf(k_supd_bf16<8, NTW, GB>, grid, dim3(512), st, pr, (const uint16_t*)X.v, X.ld, X.d,
              b, idx, Ch, Cl, ldC, PC, p, G, Dl, Dh, Dlo, ldD, lam, eta);
  });
  return hipGetLastError();
}

}  // namespace lr
