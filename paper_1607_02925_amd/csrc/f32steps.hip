// FP32 matrix-core inner steps (v_mfma_f32_16x16x4f32, FP32 accumulation) for
// dense X stored in FP32 or BF16 (exact in FP32).
//
// The instruction multiplies a 16 x 4 A by a 4 x 16 B: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], and receives D[4 (l / 16) + v][l % 16]
// in accumulator v (checked on the device).  As in the FP64 kernels, lane
// (c = l % 16, q = l / 16) of a 16-row block supplies k = 4 q + s at step s.
//
// FP32 copies of the step difference (D32) and of C (C32) are kept in 1 KB
// tiles: for each 16-row (or 16-sample) block and 16-column slice, lane l's
// four values (k = 4 q .. 4 q + 3 of column c) sit at floats 4 l .. 4 l + 3,
// so a wave reads a tile as one contiguous load.  The FP64 step difference
// stays the master: the update computes it in FP64 from the FP32-accumulated
// product and rounds it to the FP32 tile for the next step; the passes stay
// FP64, so each epoch restarts from an exactly computed residual.
//
// One X load serves every column slice (the sample dot takes all slices in a
// workgroup; so does the update once d has 256 row tiles).  For minibatches
// under 256 blocks of 16 samples the sample dot splits the rows of X over two
// workgroups that write separate partial C32 copies, which the update adds as
// it loads them: no workgroup waits on another.
#include "f32steps.h"

#include <hip/hip_ext.h>

namespace lr {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KS32 = 8192;   // largest minibatch; its indices are staged in LDS

__device__ __forceinline__ f32x4 mfma32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float xload(const float* p) { return *p; }
__device__ __forceinline__ float xload(const uint16_t* p) {
  return __uint_as_float((uint32_t)*p << 16);
}

// Float offset of (k, j) in a 1 KB-tile FP32 copy with NS 16-column slices.
__device__ __forceinline__ int64_t t32_off(int64_t k, int j, int NS) {
  const int w = (int)(k & 15);
  return (((k >> 4) * NS + (j >> 4)) * 64 + (w >> 2) * 16 + (j & 15)) * 4 + (w & 3);
}

__device__ __forceinline__ float4 tile32(const float* __restrict__ base, int64_t kb, int u, int NS,
                                         int l) {
  return *reinterpret_cast<const float4*>(base + ((kb * NS + u) * 64 + l) * 4);
}

// Four consecutive entries of one column (rows r..r+3 < d) as FP32.
template <typename TX, bool VEC>
__device__ __forceinline__ float4 load4f(const TX* __restrict__ col, int64_t r) {
  if constexpr (VEC && sizeof(TX) == 4) {
    return *reinterpret_cast<const float4*>(col + r);
  } else if constexpr (VEC) {
    const uint2 a = *reinterpret_cast<const uint2*>(col + r);
    return make_float4(__uint_as_float(a.x << 16), __uint_as_float(a.x & 0xFFFF0000u),
                       __uint_as_float(a.y << 16), __uint_as_float(a.y & 0xFFFF0000u));
  } else {
    return make_float4(xload(col + r), xload(col + r + 1), xload(col + r + 2), xload(col + r + 3));
  }
}

// The same with rows >= d read as 0 (addresses clamped to row d - 1).
template <typename TX>
__device__ __forceinline__ float4 load4ftail(const TX* __restrict__ col, int64_t r, int64_t d) {
  float v[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float x = xload(col + min(r + s, d - 1));
    v[s] = r + s < d ? x : 0.f;
  }
  return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ float f4get(const float4& v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// Orders a wave's LDS accesses around it (a wave's own LDS operations complete
// in issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum the NW waves' accumulators (NT 16x16 tiles each) into red[0 .. NT*256)
// in wave order, one tile at a time through NW*256 slots; element (i, j) of
// tile u lands at red[u * 256 + i * 16 + j].
template <int NW, int NT>
__device__ __forceinline__ void waves_sum32(double* red, double* slots, const f32x4* acc, int q,
                                            int c) {
  const int t = threadIdx.x, wave = t / 64;
  double* mine = slots + wave * 256;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) mine[(4 * q + v) * 16 + c] = (double)acc[u][v];
    __syncthreads();
    for (int e = t; e < 256; e += NW * 64) {
      double s = slots[e];
#pragma unroll
      for (int w = 1; w < NW; ++w) s += slots[w * 256 + e];
      red[u * 256 + e] = s;
    }
    __syncthreads();
  }
}

// Number of row splits of the sample dot: 2 below 256 blocks of 16 samples,
// so the workgroups cover more of the 256 compute units, else 1.  (Four splits
// cost the update more than they save the dot at every size measured.)
inline int dot_splits(int64_t b) { return (b + 15) / 16 >= 256 ? 1 : 2; }

// Partial C32 for 16 samples x all NT = PC / 16 column slices over the rows of
// split z = blockIdx.z (a run of bps 16-row blocks, possibly empty):
// C32p_z = diag(scale) X_B^T D32 restricted to those rows, at C32 + z cstride.
// One X load serves all slices.  The NW waves split the split's row blocks.
// Two register stages of G 16-row blocks; every load reads an in-bounds
// address (samples past b read column idx[0] and are written as zero rows, a
// stage's overhang re-reads the wave's last block and skips its matrix-core
// work on a wave-uniform branch, and the partial last row block is done on its
// own with clamped, zeroed X loads; the tiles of D32 hold zeros past d).
template <typename TX, int NW, int G, bool VEC, int NT>
__global__ __launch_bounds__(NW * 64) void k_sdot_f32(const TX* __restrict__ X, int64_t ld,
                                                      int64_t d, int64_t b,
                                                      const int32_t* __restrict__ idx,
                                                      const double* __restrict__ scale,
                                                      const float* __restrict__ D32,
                                                      float* __restrict__ C32, int64_t bps,
                                                      int64_t cstride) {
  __shared__ double red[NT * 256];
  __shared__ double slots[NW * 256];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, c = l % 16, q = l / 16;
  const int64_t s0 = (int64_t)blockIdx.x * 16;
  const TX* __restrict__ xcol = X + (int64_t)idx[s0 + c < b ? s0 + c : 0] * ld;
  // the epilogue's weight, loaded now so that its latency hides under the loop
  // (thread t writes rows i = (t % 256) / 16 of every slice)
  const int64_t sw = s0 + (t % 256) / 16;
  const double wsc = scale[sw < b ? sw : 0];
  f32x4 acc[NT];
#pragma unroll
  for (int v = 0; v < NT; ++v) acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nblk = (d + 15) / 16, nfull = d / 16;
  const int64_t k0 = min(nblk, (int64_t)blockIdx.z * bps), k1 = min(nblk, k0 + bps);
  const int64_t bpw = (k1 - k0 + NW - 1) / NW;
  const int64_t b0 = k0 + wave * bpw, b1 = min(k1, b0 + bpw);
  const int64_t bend = min(b1, nfull);
  struct Stage {
    float4 x[G];
    float4 m[G][NT];
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t blk = min(g + i, bend - 1);
      S.x[i] = load4f<TX, VEC>(xcol, blk * 16 + 4 * q);
#pragma unroll
      for (int v = 0; v < NT; ++v) S.m[i][v] = tile32(D32, blk, v, NT, l);
    }
  };
  auto compute = [&](const Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (g + i >= bend) break;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < NT; ++v)
          acc[v] = mfma32(f4get(S.x[i], s), f4get(S.m[i][v], s), acc[v]);
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
  if (nfull < nblk && b0 <= nfull && nfull < b1) {   // the partial last block of rows
    const float4 x = load4ftail<TX>(xcol, nfull * 16 + 4 * q, d);
#pragma unroll
    for (int v = 0; v < NT; ++v) {
      const float4 m = tile32(D32, nfull, v, NT, l);
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[v] = mfma32(f4get(x, s), f4get(m, s), acc[v]);
    }
  }
  waves_sum32<NW, NT>(red, slots, acc, q, c);
  // rows from b up to the next multiple of 16 are written as zeros (the update
  // reads whole 16-sample blocks)
  float* __restrict__ out = C32 + (int64_t)blockIdx.z * cstride;
  static_assert((NW * 64) % 256 == 0, "a thread keeps its row i across slices");
  for (int e = t; e < NT * 256; e += NW * 64) {
    const int v = e / 256, i = (e % 256) / 16, j = e % 16;
    const int64_t ss = s0 + i;
    out[t32_off(ss, v * 16 + j, NT)] = ss < b ? (float)(wsc * red[e]) : 0.f;
  }
}

// Dl <- Dl - eta (G + lam Dl - U), U[r, j] = sum_s X[r, idx[s]] C[s, j] with C
// the sum of the KS partial copies at C32 + z cstride, for a tile of 16 rows
// and NT column slices starting at slice NT blockIdx.y (one X load serves
// them all); the new Dl (FP64, tile-major, the layout of the FP64 path) is
// also rounded into the FP32 tile for the next step.  The NW waves split the
// samples (indices staged in LDS, padded to a multiple of 16 with a valid
// column; C32 holds zero rows past b); two register stages.  A block of 16
// samples is fetched with one load per lane: lane l takes rows 4 (l % 4) ..
// + 3 of the tile from sample l / 4 (16 contiguous bytes of FP32 X, 8 of
// BF16 X; VEC moves a piece past d back to rows d - 4 .. d - 1, the scalar
// form reads rows past d as zero), and the wave turns the 16 x 16 block
// around through its own LDS tile (two, alternating) into the matrix-core
// operand order, row c and samples 4 q .. 4 q + 3 for lane 16 q + c.  Rows
// past d are not stored.  The grid (a multiple of 8 tiles) is remapped so each XCD owns a
// contiguous run of row tiles.
template <typename TX, int NW, int G, int NT, int KS, bool VEC>
__global__ __launch_bounds__(NW * 64) void k_supd_f32(const TX* __restrict__ X, int64_t ld,
                                                      int64_t d, int64_t b,
                                                      const int32_t* __restrict__ idx,
                                                      const float* __restrict__ C32,
                                                      int64_t cstride, int p, int NS,
                                                      const double* __restrict__ Gr,
                                                      double* __restrict__ Dl,
                                                      float* __restrict__ D32, double lam,
                                                      double eta) {
  constexpr int XTP = 20;   // pitch of a transpose tile: the 64 lanes' writes meet 64 banks
  __shared__ double red[NT * 256];
  __shared__ double slots[NW * 256];
  __shared__ int sidx[KS32];
  __shared__ __align__(16) float xtr[NW][2][16 * XTP];
  const int t = threadIdx.x, wave = t / 64, l = t % 64, c = l % 16, q = l / 16;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  const int64_t r0 = tile * 16;
  if (r0 >= d) return;
  const int u0 = blockIdx.y * NT;
  // thread t < NT * 256 updates element (r0 + (t % 256) / 16, column (u0 + t / 256) 16 + t % 16)
  // in the epilogue; its FP64 operands are loaded now so that their latency
  // hides under the loop (an element past d or p reads element 0 and is not stored)
  static_assert(NW * 64 >= NT * 256, "one element per thread");
  const int ei = (t % 256) / 16, ej = (u0 + t / 256) * 16 + t % 16;
  const int64_t er = r0 + ei;
  const bool eown = t < NT * 256 && er < d && ej < p;
  int64_t eo = 0;
  if (eown) {
    const int rho = (int)(er & 15), qq = rho >> 2, ss = rho & 3;
    eo = ((er >> 4) * NS + (ej >> 4)) * 256 + (ss >> 1) * 128 + (qq * 16 + (ej & 15)) * 2 + (ss & 1);
  }
  const double edl = Dl[eo];
  const double egr = Gr[eown ? (int64_t)ej * d + er : 0];
  const int64_t bpad = (b + 15) / 16 * 16;
  for (int64_t e = t; e < bpad; e += NW * 64) sidx[e] = idx[e < b ? e : 0];
  __syncthreads();
  const int lj = l >> 2, lr = 4 * (l & 3);   // this lane's sample and first row in a block
  const int64_t rr = r0 + lr;
  const int64_t rl = VEC && rr + 4 > d ? d - 4 : rr;
  f32x4 acc[NT];
#pragma unroll
  for (int v = 0; v < NT; ++v) acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t nblk = bpad / 16;
  const int64_t bpw = (nblk + NW - 1) / NW;
  const int64_t b0 = wave * bpw, b1 = min(nblk, b0 + bpw);
  struct Stage {
    float4 x[G];
    float4 m[G][NT][KS];   // the partials of C, added where they are used
  };
  auto load = [&](Stage& S, int64_t g) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int64_t blk = min(g + i, b1 - 1);
      const TX* __restrict__ col = X + (int64_t)sidx[blk * 16 + lj] * ld;
      S.x[i] = VEC ? load4f<TX, true>(col, rl) : load4ftail<TX>(col, rr, d);
#pragma unroll
      for (int v = 0; v < NT; ++v)
#pragma unroll
        for (int z = 0; z < KS; ++z) S.m[i][v][z] = tile32(C32 + z * cstride, blk, u0 + v, NS, l);
    }
  };
  auto compute = [&](const Stage& S, int64_t g, bool checked) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      if (checked && g + i >= b1) break;
      float* __restrict__ wt = xtr[wave][(g + i) & 1];
      wt[(lr + 0) * XTP + lj] = S.x[i].x;
      wt[(lr + 1) * XTP + lj] = S.x[i].y;
      wt[(lr + 2) * XTP + lj] = S.x[i].z;
      wt[(lr + 3) * XTP + lj] = S.x[i].w;
      wave_sync();
      const float4 a = *reinterpret_cast<const float4*>(wt + c * XTP + 4 * q);
      wave_sync();
      float4 cm[NT];
#pragma unroll
      for (int v = 0; v < NT; ++v) {
        cm[v] = S.m[i][v][0];
#pragma unroll
        for (int z = 1; z < KS; ++z) {
          cm[v].x += S.m[i][v][z].x;
          cm[v].y += S.m[i][v][z].y;
          cm[v].z += S.m[i][v][z].z;
          cm[v].w += S.m[i][v][z].w;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < NT; ++v) acc[v] = mfma32(f4get(a, s), f4get(cm[v], s), acc[v]);
    }
  };
  if (b0 < b1) {
    // whole pairs of stages first, with no branch between a stage's loads and
    // the work before its use (a guarded use would let the compiler move the
    // loads down to it, and the next stage's loads would no longer overlap)
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
  waves_sum32<NW, NT>(red, slots, acc, q, c);
  if (eown) {
    // the FP64 master, tile-major as on the FP64 path
    const double x = edl - eta * (egr + lam * edl - red[t]);
    Dl[eo] = x;
    D32[t32_off(er, ej, NS)] = (float)x;
  }
}

template <typename K, typename... A>
static void launch32(K kernel, dim3 grid, dim3 block, hipStream_t st, const Probe& pr, A... args) {
  if (pr.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pr.start, pr.stop, 0, args...);
  else
    kernel<<<grid, block, 0, st>>>(args...);
}

template <typename TX, bool VEC, int NT>
void sdot_launch(const XView& X, int64_t b, const int32_t* idx, const double* scale,
                 const float* D32, float* C32, hipStream_t st, const Probe& pr, int ks) {
  const int64_t nblk = (X.d + 15) / 16;
  const dim3 grid((unsigned)((b + 15) / 16), 1, (unsigned)ks);
  // four waves per workgroup: 4-7% faster than eight at d = 2048 and 4096
  launch32(k_sdot_f32<TX, 4, 2, VEC, NT>, grid, dim3(256), st, pr, (const TX*)X.v, X.ld, X.d, b,
           idx, scale, D32, C32, (nblk + ks - 1) / ks, (b + 15) / 16 * 16 * (NT * 16));
}

template <typename TX, bool VEC>
void sdot_nt(int NS, const XView& X, int64_t b, const int32_t* idx, const double* scale,
             const float* D32, float* C32, hipStream_t st, const Probe& pr, int ks) {
  switch (NS) {
    case 1: sdot_launch<TX, VEC, 1>(X, b, idx, scale, D32, C32, st, pr, ks); break;
    case 2: sdot_launch<TX, VEC, 2>(X, b, idx, scale, D32, C32, st, pr, ks); break;
    case 3: sdot_launch<TX, VEC, 3>(X, b, idx, scale, D32, C32, st, pr, ks); break;
    default: sdot_launch<TX, VEC, 4>(X, b, idx, scale, D32, C32, st, pr, ks); break;
  }
}

// Row tiles of 16 from which the update takes all column slices in one
// workgroup (fewer tiles: one slice per workgroup, so the grid still covers
// the compute units).
constexpr int64_t UPD_ALL_SLICES_TILES = 256;

template <typename TX, int NT, int KS>
void supd_launch(const XView& X, int p, int NS, int64_t b, const int32_t* idx, const float* C32,
                 const double* G, double* Dl, float* D32, double lam, double eta, hipStream_t st,
                 const Probe& pr) {
  const dim3 grid((unsigned)(((X.d + 15) / 16 + 7) / 8 * 8), (unsigned)(NS / NT));
  // 16-byte (FP32) or 8-byte (BF16) pieces of 4 rows: aligned columns, d a multiple of 4
  const bool vec = X.ld % 4 == 0 && X.d % 4 == 0 && (uintptr_t)X.v % (4 * sizeof(TX)) == 0;
  if (vec)
    launch32(k_supd_f32<TX, 16, 1, NT, KS, true>, grid, dim3(1024), st, pr, (const TX*)X.v, X.ld,
             X.d, b, idx, C32, (b + 15) / 16 * 16 * (NS * 16), p, NS, G, Dl, D32, lam, eta);
  else
    launch32(k_supd_f32<TX, 16, 1, NT, KS, false>, grid, dim3(1024), st, pr, (const TX*)X.v, X.ld,
             X.d, b, idx, C32, (b + 15) / 16 * 16 * (NS * 16), p, NS, G, Dl, D32, lam, eta);
}

template <typename TX, int KS>
void supd_nt(int NS, const XView& X, int p, int64_t b, const int32_t* idx, const float* C32,
             const double* G, double* Dl, float* D32, double lam, double eta, hipStream_t st,
             const Probe& pr) {
  switch ((X.d + 15) / 16 >= UPD_ALL_SLICES_TILES ? NS : 1) {
    case 2: supd_launch<TX, 2, KS>(X, p, NS, b, idx, C32, G, Dl, D32, lam, eta, st, pr); break;
    case 3: supd_launch<TX, 3, KS>(X, p, NS, b, idx, C32, G, Dl, D32, lam, eta, st, pr); break;
    case 4: supd_launch<TX, 4, KS>(X, p, NS, b, idx, C32, G, Dl, D32, lam, eta, st, pr); break;
    default: supd_launch<TX, 1, KS>(X, p, NS, b, idx, C32, G, Dl, D32, lam, eta, st, pr); break;
  }
}

template <typename TX>
void supd_ks(int NS, const XView& X, int p, int64_t b, const int32_t* idx, const float* C32,
             const double* G, double* Dl, float* D32, double lam, double eta, hipStream_t st,
             const Probe& pr, int ks) {
  if (ks == 1)
    supd_nt<TX, 1>(NS, X, p, b, idx, C32, G, Dl, D32, lam, eta, st, pr);
  else
    supd_nt<TX, 2>(NS, X, p, b, idx, C32, G, Dl, D32, lam, eta, st, pr);
}

}  // namespace

hipError_t step_dot_f32(const XView& X, int p, int64_t b, const int32_t* idx,
                        const double* scale, const float* D32, float* C32, int PC,
                        hipStream_t st, const Probe& pr) {
  if ((X.dt != 1 && X.dt != 2) || b < 1 || PC % 16 || PC > 64 || p > PC || PC - p >= 16 ||
      (uintptr_t)D32 % 16 || (uintptr_t)C32 % 16)
    return hipErrorInvalidValue;
  const bool vec = X.dt == 1 ? X.ld % 4 == 0 && (uintptr_t)X.v % 16 == 0
                             : X.ld % 4 == 0 && (uintptr_t)X.v % 8 == 0;
  const int NS = PC / 16;
  if (X.dt == 1) {
    if (vec)
      sdot_nt<float, true>(NS, X, b, idx, scale, D32, C32, st, pr, dot_splits(b));
    else
      sdot_nt<float, false>(NS, X, b, idx, scale, D32, C32, st, pr, dot_splits(b));
  } else {
    if (vec)
      sdot_nt<uint16_t, true>(NS, X, b, idx, scale, D32, C32, st, pr, dot_splits(b));
    else
      sdot_nt<uint16_t, false>(NS, X, b, idx, scale, D32, C32, st, pr, dot_splits(b));
  }
  return hipGetLastError();
}

hipError_t step_update_f32(const XView& X, int p, int64_t b, const int32_t* idx, const float* C32,
                           int PC, const double* G, double* Dl, float* D32, double lam,
                           double eta, hipStream_t st, const Probe& pr) {
  if ((X.dt != 1 && X.dt != 2) || b < 1 || b > KS32 || PC % 16 || PC > 64 || p > PC ||
      PC - p >= 16 || (uintptr_t)C32 % 16)
    return hipErrorInvalidValue;
  const int NS = PC / 16;
  if (X.dt == 1)
    supd_ks<float>(NS, X, p, b, idx, C32, G, Dl, D32, lam, eta, st, pr, dot_splits(b));
  else
    supd_ks<uint16_t>(NS, X, p, b, idx, C32, G, Dl, D32, lam, eta, st, pr, dot_splits(b));
  return hipGetLastError();
}

}  // namespace lr
