// Launchers of the compressed-column (CSC) kernels.  X is d x n with column i
// stored in entries [cp[i], cp[i+1]) of (ri, v): row ids sorted and distinct
// within each column, values of dtype `dt` (0 f64, 1 f32, 2 bf16 bits).  Dense
// d x p blocks are FP64; "row-major" blocks hold row r at [r * PC, r * PC + PC)
// with columns >= p zero.  Every launcher enqueues on `st` and returns
// hipSuccess or the launch error.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace lr {

struct CscView {
  const void* v;
  const int32_t* cp;
  const int32_t* ri;
  int64_t d, n, nnz;
  int dt;
};

// The row-ordered copy of X built once per plan: entries of row r at
// [row_ptr[r], row_ptr[r+1]) of (col, val), columns ascending.  Rows are cut
// into chunks of at most SP_CHUNK entries: chunk c covers entries
// [chunk_beg[c], chunk_beg[c+1]), row r owns chunks [row_chunk[r], row_chunk[r+1]).
struct CsrView {
  const int32_t* col;
  const void* val;
  const int32_t* chunk_beg;
  const int32_t* row_chunk;
  int64_t d, nch;
  int dt;
};
constexpr int SP_CHUNK = 2048;
// Most contributions (minibatch x the most entries any column stores) for
// which a plan keeps the buffers of the inner step's sorted scatter.
constexpr int64_t SP_SORT_CAP = (int64_t)1 << 22;

// Structure checks (flags OR-ed into *bad): 1 = col_ptr not a non-decreasing
// sequence from 0 to nnz; 2 = a row id outside [0, d) or not increasing within
// its column.  csc_check_rows may only run once csc_check_ptr has passed.
hipError_t csc_check_ptr(const CscView& X, int* bad, hipStream_t st);
hipError_t csc_check_rows(const CscView& X, int* bad, hipStream_t st);
// w_i = sum of squares of column i's stored values in row order, FP64, no fused
// multiply-add (the same roundings as the dense row-order sum); NaN/Inf flag.
hipError_t csc_colnorms(const CscView& X, double* w, int* bad, hipStream_t st);

// Transpose to rows: stable radix sort of the row ids (temp from csr_sort_bytes),
// then row_ptr (d + 1), col and val (nnz each).
hipError_t csr_sort_bytes(int64_t nnz, int64_t d, size_t* bytes);
hipError_t csr_build(const CscView& X, void* temp, size_t temp_bytes, uint32_t* keys_out,
                     int32_t* pos_in, int32_t* pos_out, int32_t* row_ptr, int32_t* col,
                     void* val, hipStream_t st);

// Layout changes between column-major d x ncols (ld d) and row-major d x PC.
hipError_t cm_to_rm(const double* W, int64_t d, int ncols, double* Wrm, int PC, hipStream_t st);
hipError_t rm_to_cm(const double* Wrm, int64_t d, int ncols, int PC, double* W, hipStream_t st);

// Pass, first half: T[i * PC + j] = sum_k v_k Wrm[r_k * PC + j] over column i.
hipError_t csc_xtw(const CscView& X, const double* Wrm, int PC, double* T, hipStream_t st,
                   const Probe& pr = Probe());
// Pass, second half: out = alpha X T + beta A + gamma B (d x p column-major),
// through the row-ordered copy: chunk partial sums (part: nch x PC), then each
// row's chunks in order.
hipError_t csr_xt(const CsrView& R, const double* T, int PC, int p, double* part, double alpha,
                  const double* A, double beta, const double* B, double gamma, double* out,
                  hipStream_t st, const Probe& pr = Probe());

// Inner step, part 1: C[j * PC + c] = scale_j sum_k v_k Dlrm[r_k * PC + c]
// over the stored entries of column idx[j].
hipError_t csc_step_dot(const CscView& X, int64_t b, const int32_t* idx, const double* scale,
                        const double* Dlrm, double* C, int PC, hipStream_t st,
                        const Probe& pr = Probe());
// Inner step, part 2a: Dlrm <- Dlrm - eta (Grm + lam Dlrm) elementwise.
hipError_t rm_decay(int64_t count, const double* Grm, double* Dlrm, double lam, double eta,
                    hipStream_t st);
// Inner step, part 2b: Dlrm[r, c] += eta sum_j X[r, idx[j]] C[j, c], c < p.
// Rows with head_slot[r] >= 0 (head_row[slot] = r, slot < H) are summed per
// workgroup in LDS first; all additions to Dlrm are FP64 atomics (used when
// the sorted form's buffers would exceed the plan's cap).
int sp_head_cap(int PC);
// Inner step, part 2b in a fixed order: the b maxnnz contributions (maxnnz: the
// most entries any column stores) sorted by row with a stable radix sort, each
// row's run summed in sample order; no atomics, so the result does not depend
// on timing.  Device buffers for up to total_max contributions:
struct SpSortBufs {
  uint32_t *keys_in, *keys_out;   // total_max each
  int32_t *pos_in, *pos_out;      // total_max each
  double* xval;                   // total_max: each contribution's stored value
  int32_t* hist;                  // 256 x (sp_sort_tiles(total_max) + 1): counts, totals
  double* carry;                  // sp_chunks(total_max) x 2 x PC
  int32_t* flags;                 // sp_chunks(total_max)
  int64_t total_max;
};
int64_t sp_chunks(int64_t total);
int64_t sp_sort_tiles(int64_t total);
// All device bytes of SpSortBufs for total_max contributions.
size_t sp_sort_bytes(int64_t total_max, int PC);
hipError_t csc_step_scatter_sorted(const CscView& X, int64_t b, int maxnnz, const int32_t* idx,
                                   const double* C, int PC, int p, double eta,
                                   const SpSortBufs& sb, double* Dlrm, hipStream_t st,
                                   const Probe& pr = Probe());
hipError_t csc_step_scatter(const CscView& X, int64_t b, const int32_t* idx, const double* C,
                            int PC, int p, const int32_t* head_slot, const int32_t* head_row,
                            int H, double eta, double* Dlrm, hipStream_t st,
                            const Probe& pr = Probe());

}  // namespace lr
