// Host engine of the shift-and-invert low-rank path and the C ABI of
// lowrank.h.  The engine only sequences device kernels and takes the scalar
// decisions of the method (gap budget, shift, inner-solver constants, stopping)
// from small device-to-host copies; every step over X or a d x p block runs
// on the GPU.
#include "lowrank.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "engine.h"
#include "bf16.h"
#include "f32steps.h"
#include "kernels.h"
#include "mcpass.h"
#include "sparse.h"

namespace {

thread_local std::string g_err;

lr_status fail(lr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define LR_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LR_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define LR_CHECK(expr)              \
  do {                              \
    lr_status s_ = (expr);          \
    if (s_ != LR_OK) return s_;     \
  } while (0)

constexpr uint32_t TAG_EST_INIT = 1, TAG_SI_INIT = 2, TAG_SAMPLES = 3, TAG_POWER_INIT = 4;

inline uint32_t stream_word(uint32_t tag, uint32_t solve) { return (tag << 28) | solve; }

}  // namespace

namespace lr {
void set_last_error(const std::string& msg) { g_err = msg; }
std::string last_error() { return g_err; }
}  // namespace lr

struct lr_plan_s {
  hipStream_t st = nullptr;
  lr::XView X{};
  // compressed-column X: the caller's CSC view, the row-ordered copy built at
  // plan time (owned, separate allocations) and the row-major d x PC blocks
  bool sparse = false;
  lr::CscView Xs{};
  lr::CsrView R{};
  std::vector<void*> sp_allocs;
  int32_t *sp_head_slot = nullptr, *sp_head_row = nullptr;
  int sp_H = 0;
  double* sp_part = nullptr;
  // the inner step's scatter in a fixed order (sp_sorted), for up to
  // bmax x sp_maxnnz contributions
  bool sp_sorted = false;
  int sp_maxnnz = 0;
  lr::SpSortBufs sp_sb{};
  double *Wrm = nullptr, *Grm = nullptr, *Dlrm = nullptr;
  // BF16 matrix-core inner steps: split copies of the difference block (ldD x PC)
  // and of the sampled products (PC x ldC)
  bool bf16_steps = false;
  int64_t ldD = 0, ldC = 0;
  // FP32 matrix-core inner steps: FP32 tile copies of the difference block
  // (pad16(d) x PC) and of the sampled products (up to 2 partial sums over row
  // ranges, each pad16(bmax) x PC)
  bool f32_steps = false;
  float *D32 = nullptr, *C32 = nullptr;
  // matrix-core passes (FP32 / BF16 X): BF16 parts of W and T, FP32 partial
  // sums; used by the passes of the shift-and-invert solves while mc_active
  bool mc_pass = false, mc_active = false;
  lr::McBufs mb{};
  // adaptive partitioning (Algorithm "main"): the deflation basis Ud (d x ns),
  // Z = X^T Ud (n x pad16(ns) row-major), projection temporaries, the chunk
  // partials of the deflated inner step
  bool adaptive = false;
  // accelerated inner solver: the next iterate, two momentum points, the shifted
  // right-hand side S + kappa Y
  bool accel = false;
  double acc_kappa = 0.0, acc_beta = 0.0;   // of the shift-and-invert solves
  double *Wn = nullptr, *Ya = nullptr, *Yb = nullptr, *Racc = nullptr;
  int ns = 0;
  double *Ud = nullptr, *Zt = nullptr, *Dw1 = nullptr, *Dw2 = nullptr, *Kd = nullptr, *Vp = nullptr;
  uint16_t *Dh = nullptr, *Dlo = nullptr, *Ch = nullptr, *Cl = nullptr;
  int k = 0, p = 0;
  double eps = 0;
  lr_options opt{};
  bool replay = false;
  lr_schedule rsched{};
  std::vector<int32_t> repochs;
  int64_t d = 0, n = 0, bmax = 0;
  int PC = 0;                     // padded row stride of T and C
  static constexpr int64_t MCH = 256;  // inner steps whose draws are made in one launch

  void* ws = nullptr;              // the one device block all buffers are carved from
  bool owns_ws = true;             // false: the block belongs to a server arena
  bool owns_host = true;           // false: hpin and ev belong to a server slot
  double *w = nullptr, *S = nullptr, *W = nullptr, *Wt = nullptr, *G = nullptr, *Y = nullptr;
  double *Wtl = nullptr;   // tile-major copy of the pass operand (dense X)
  double *Dl = nullptr, *Tm1 = nullptr, *Tm2 = nullptr, *Sest = nullptr, *V = nullptr;
  double *Vprev = nullptr, *T = nullptr, *Ypart = nullptr, *C = nullptr, *scale = nullptr;
  double *part = nullptr, *scratch = nullptr;
  double *H = nullptr, *Q = nullptr, *vals = nullptr, *M = nullptr, *Rinv = nullptr;
  double *kk1 = nullptr, *kk2 = nullptr, *res = nullptr, *dfro2 = nullptr, *dnorm = nullptr;
  uint64_t* cdf = nullptr;
  int32_t* idx = nullptr;
  int *dinfo = nullptr, *dbad = nullptr;
  double* hpin = nullptr;
  lr::PassBufs pb{};
  hipEvent_t ev[8] = {};

  bool prepared = false;
  double fro2 = 0;
  lr_schedule sched{};
  std::vector<int32_t> epochs;
  lr_report rep{};

  ~lr_plan_s() {
    for (void* a : sp_allocs) (void)hipFree(a);
    if (owns_ws && ws) (void)hipFree(ws);
    if (owns_host) {
      if (hpin) (void)hipHostFree(hpin);
      for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    }
  }

  // Lay every device buffer out in one block at `base` (256-byte aligned
  // pieces); with base == nullptr only the total size is computed.
  size_t carve(char* base);

  // Copy `bytes` from device to host (synchronises the stream).
  lr_status read(void* host, const void* dev, size_t bytes) {
    LR_HIP(hipMemcpyAsync(hpin, dev, bytes, hipMemcpyDeviceToHost, st));
    LR_HIP(hipStreamSynchronize(st));
    std::memcpy(host, hpin, bytes);
    return LR_OK;
  }

  lr_status check_spd() {
    int info = 0;
    LR_CHECK(read(&info, dinfo, sizeof(int)));
    if (info) return fail(LR_ENOTSPD, "Cholesky-QR: Gram matrix not positive definite");
    return LR_OK;
  }

  // T = X^T W (n x PC row-major)   (W: d x ncols)
  lr_status xtw(const double* Win, int ncols) {
    if (sparse) {
      LR_HIP(lr::cm_to_rm(Win, d, ncols, Wrm, PC, st));
      LR_HIP(lr::csc_xtw(Xs, Wrm, PC, T, st));
    } else {
      LR_HIP(lr::pass_xtw(X, Win, ncols, T, PC, Wtl, st));
    }
    return LR_OK;
  }

  // Y = alpha X (X^T W) + beta A + gamma B   (W: d x ncols)
  // Wout = (I - Ud Ud^T) Win for the ns directions found so far (Wout may be Win)
  lr_status deflate(const double* Win, double* Wout, int ncols) {
    LR_HIP(lr::gram(Ud, 1, d, ns, Win, 1, d, ncols, d, part, Kd, st));
    LR_HIP(lr::lincomb((int64_t)ns * ncols, -1.0, Kd, 0.0, nullptr, 0.0, nullptr, Kd, st));
    LR_HIP(lr::gemm_small(d, ns, ncols, Ud, Kd, ns, Wout, 1.0, Win, st));
    return LR_OK;
  }

  // With directions found (ns > 0) the operator is the deflated A_{-(s-1)} = P A P.
  lr_status applyA(const double* Win, double* Yout, int ncols, double alpha = 1.0,
                   const double* A = nullptr, double beta = 0.0, const double* B = nullptr,
                   double gamma = 0.0) {
    if (ns > 0) {
      LR_CHECK(deflate(Win, Dw1, ncols));
      LR_CHECK(xtw(Dw1, ncols));
      LR_HIP(lr::pass_xt(X, T, PC, ncols, pb, 1.0, nullptr, 0.0, nullptr, 0.0, Dw2, st));
      LR_CHECK(deflate(Dw2, Dw1, ncols));
      LR_HIP(lr::lincomb(d * ncols, alpha, Dw1, beta, A, gamma, B, Yout, st));
      rep.passes++;
      return LR_OK;
    }
    if (mc_active && !sparse) {
      LR_HIP(lr::mc_pass(X, Win, ncols, PC, mb, alpha, A, beta, B, gamma, Yout, st));
      rep.passes++;
      rep.mc_passes++;
      return LR_OK;
    }
    LR_CHECK(xtw(Win, ncols));
    if (sparse)
      LR_HIP(lr::csr_xt(R, T, PC, ncols, sp_part, alpha, A, beta, B, gamma, Yout, st));
    else
      LR_HIP(lr::pass_xt(X, T, PC, ncols, pb, alpha, A, beta, B, gamma, Yout, st));
    rep.passes++;
    return LR_OK;
  }

  lr_status sparse_setup();
  lr_status device_structure(int* bad);
  lr_status confirm_structure(int device_flag);

  lr_status gram_dd(const double* A, int pa, const double* B, int pb_, double* out) {
    LR_HIP(lr::gram(A, 1, d, pa, B, 1, d, pb_, d, part, out, st));
    return LR_OK;
  }

  // S = W R^{-1}, twice (Cholesky-QR2).  Win may equal Sout.
  lr_status cholqr2(const double* Win, double* Sout, int ncols) {
    LR_CHECK(gram_dd(Win, ncols, Win, ncols, H));
    LR_HIP(lr::chol_rinv(H, ncols, Rinv, dinfo, st));
    LR_HIP(lr::gemm_small(d, ncols, ncols, Win, Rinv, ncols, Tm1, 0.0, nullptr, st));
    LR_CHECK(gram_dd(Tm1, ncols, Tm1, ncols, H));
    LR_HIP(lr::chol_rinv(H, ncols, Rinv, dinfo, st));
    LR_HIP(lr::gemm_small(d, ncols, ncols, Tm1, Rinv, ncols, Sout, 0.0, nullptr, st));
    return LR_OK;
  }

  lr_status prepare() {
    LR_HIP(hipMemsetAsync(dbad, 0, sizeof(int), st));
    if (sparse)
      LR_HIP(lr::csc_colnorms(Xs, w, dbad, st));
    else
      LR_HIP(lr::colnorms(X, w, dbad, st));
    int bad = 0;
    LR_CHECK(read(&bad, dbad, sizeof(int)));
    if (bad) return fail(LR_EINVAL, "non-finite entries in X");
    LR_HIP(lr::build_table(w, n, cdf, dfro2, scratch, st));
    LR_CHECK(read(&fro2, dfro2, sizeof(double)));
    if (!(fro2 > 0)) return fail(LR_EINVAL, "X is zero");
    prepared = true;
    return LR_OK;
  }

  void constants(double theta1, double lam, double mu, int64_t* b, double* eta, int64_t* m) const {
    int64_t bb;
    if (opt.batch > 0) {
      bb = opt.batch;
    } else {
      const double bstar = 4.0 * fro2 * theta1 / (lam * mu);
      const double l2 = std::ceil(std::log2(std::max(bstar, 1.0)));
      bb = (int64_t)1 << (int64_t)std::max(0.0, l2);
      bb = std::min<int64_t>(std::max<int64_t>(bb, 256), 8192);
    }
    bb = std::min(bb, n);
    const double sig2 = fro2 * theta1 / (double)bb;
    *eta = opt.eta_scale * std::min(1.0 / lam, mu / (4.0 * sig2));
    *m = (int64_t)std::ceil(2.0 / (*eta * mu));
    *b = bb;
  }

  // Constants of the inner solver for shift lam and strong-convexity estimate
  // mu.  Accelerated (opt.accel): kappa = max(0, sqrt(8 ||X||_F^2 theta_1 / n) - mu),
  // beta = (1 - sqrt(q)) / (1 + sqrt(q)) with q = mu / (mu + kappa), and the plain
  // constants taken at lam + kappa, mu + kappa.
  struct Inner {
    int64_t b = 0, m = 0;
    double eta = 0, kappa = 0, beta = 0;
  };
  Inner inner_constants(double theta1, double lam, double mu) const {
    Inner c;
    if (accel) {
      c.kappa = std::max(0.0, std::sqrt(8.0 * fro2 * theta1 / (double)n) - mu);
      const double q = mu / (mu + c.kappa);
      c.beta = (1.0 - std::sqrt(q)) / (1.0 + std::sqrt(q));
    }
    constants(theta1, lam + c.kappa, mu + c.kappa, &c.b, &c.eta, &c.m);
    return c;
  }

  // Inner solve of (lam I - XX^T) W = Srhs; the result is left in Wt.
  // kappa > 0 or accel: the accelerated proximal-point loop, one SVRG epoch on
  // ((lam + kappa) I - XX^T) W = Srhs + kappa Y per outer step, started at the
  // previous iterate; the residual is that of the original system.
  lr_status svrg_solve(const double* Srhs, double lam, double eta, int64_t m, int64_t b,
                       int32_t solve, double tau, int32_t fixed_epochs, int32_t* epochs_out,
                       std::vector<double>* hist, int ncols = -1, double kappa = 0.0,
                       double beta = 0.0) {
    if (b > bmax) return fail(LR_EINVAL, "minibatch larger than the plan's workspace");
    const int pc = ncols < 0 ? p : ncols;           // right-hand sides in this solve
    const int PCn = lr::pad16(pc);                  // row stride of C
    const int64_t cnt = d * pc;
    lr::Deflation df;
    if (ns > 0) {
      df.ns = ns;
      df.PCZ = lr::pad16(ns);
      df.nks = lr::zbc_chunks(b);
      df.Z = Zt;
      df.Ud = Ud;
      df.Vp = Vp;
    }
    // warm start W0 = S (lam I - S^T A S)^{-1}; its gradient costs no extra pass.
    // With matrix-core passes this pass stays FP64 and each epoch's pass is
    // applied to the epoch's step difference only (see the epoch update below).
    const bool mc = mc_active && !accel && ns == 0;
    mc_active = false;
    const lr_status s0 = applyA(Srhs, Y, pc);
    mc_active = mc;
    LR_CHECK(s0);
    LR_CHECK(gram_dd(Srhs, pc, Y, pc, H));
    LR_HIP(lr::eigh(H, pc, vals, Q, st));
    LR_HIP(lr::shift_inverse(vals, Q, pc, lam, M, st));
    LR_HIP(lr::gemm_small(d, pc, pc, Srhs, M, pc, Wt, 0.0, nullptr, st));
    LR_HIP(lr::lincomb(cnt, lam, Srhs, -1.0, Y, 0.0, nullptr, Tm1, st));
    LR_HIP(lr::gemm_small(d, pc, pc, Tm1, M, pc, G, -1.0, Srhs, st));
    LR_HIP(lr::sumsq(Srhs, cnt, part, dnorm, st));
    LR_HIP(lr::sumsq(G, cnt, part, dnorm + 1, st));
    double nr[2];
    LR_CHECK(read(nr, dnorm, 2 * sizeof(double)));
    const double sn = std::sqrt(nr[0]);
    const double r0 = std::sqrt(nr[1]);
    double r = r0;
    if (hist) hist->push_back(r);
    const uint32_t w3 = stream_word(TAG_SAMPLES, (uint32_t)solve);
    const double lam_in = lam + kappa;   // the steps' shift
    const bool tiled = !sparse && !bf16_steps;   // Dl tile-major (dense FP64 steps)
    double* Yk = Ya;
    double* Ynew = Yb;
    if (accel)   // Y_0 = W_0; the inner gradient at W_0 equals the original one
      LR_HIP(hipMemcpyAsync(Yk, Wt, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (bf16_steps) {   // sample slots beyond b stay zero for the whole solve
      LR_HIP(hipMemsetAsync(Ch, 0, ldC * PC * sizeof(uint16_t), st));
      LR_HIP(hipMemsetAsync(Cl, 0, ldC * PC * sizeof(uint16_t), st));
    }
    // an accelerated outer step gains about 1 - sqrt(q) where a plain epoch gains a
    // constant factor: its budget is max_epochs ceil(1 / sqrt(q)), 1 / sqrt(q) = (1 + beta) / (1 - beta)
    const int64_t budget =
        accel ? (int64_t)opt.max_epochs * (int64_t)std::ceil((1.0 + beta) / (1.0 - beta))
              : (int64_t)opt.max_epochs;
    int32_t e = 0;
    for (;;) {
      if (fixed_epochs < 0) {
        if (r <= tau * sn) break;
        if (e >= budget) return fail(LR_ENOCONV, "inner solver did not converge");
      } else if (e >= fixed_epochs) {
        break;
      }
      if (sparse) {
        LR_HIP(lr::cm_to_rm(G, d, p, Grm, PC, st));
        LR_HIP(hipMemsetAsync(Dlrm, 0, d * PC * sizeof(double), st));
      } else {
        LR_HIP(hipMemsetAsync(Dl, 0, (tiled ? lr::pad16(d) * PCn : cnt) * sizeof(double), st));
        if (bf16_steps) {
          LR_HIP(hipMemsetAsync(Dh, 0, ldD * PC * sizeof(uint16_t), st));
          LR_HIP(hipMemsetAsync(Dlo, 0, ldD * PC * sizeof(uint16_t), st));
        }
        if (f32_steps) LR_HIP(hipMemsetAsync(D32, 0, lr::pad16(d) * PC * sizeof(float), st));
      }
      if (opt.timing) LR_HIP(hipEventRecord(ev[0], st));
      const int64_t tprobe = m / 2;  // one launch per epoch is timed per kernel
      for (int64_t t0 = 0; t0 < m; t0 += MCH) {
        const int64_t nst = std::min(MCH, m - t0);
        LR_HIP(lr::draw_chunk(n, cdf, opt.seed, (uint32_t)t0, nst, (uint32_t)e, w3, b, idx, scale,
                              st));
        for (int64_t t = t0; t < t0 + nst; ++t) {
          const bool probe = opt.timing && t == tprobe;
          const int32_t* it = idx + (t - t0) * b;
          lr::Probe pd, pu;
          if (probe) {
            pd.start = ev[4];
            pd.stop = ev[5];
            pu.start = ev[6];
            pu.stop = ev[7];
          }
          if (sparse) {
            LR_HIP(lr::csc_step_dot(Xs, b, it, scale + (t - t0) * b, Dlrm, C, PC, st, pd));
            LR_HIP(lr::rm_decay(d * PC, Grm, Dlrm, lam_in, eta, st));
            if (sp_sorted)
              LR_HIP(lr::csc_step_scatter_sorted(Xs, b, sp_maxnnz, it, C, PC, p, eta, sp_sb,
                                                 Dlrm, st, pu));
            else
              LR_HIP(lr::csc_step_scatter(Xs, b, it, C, PC, p, sp_head_slot, sp_head_row, sp_H,
                                          eta, Dlrm, st, pu));
          } else if (bf16_steps) {
            LR_HIP(lr::step_dot_bf16(X, p, b, it, scale + (t - t0) * b, Dh, Dlo, ldD, Ch, Cl,
                                     ldC, PC, st, pd));
            LR_HIP(lr::step_update_bf16(X, p, b, it, Ch, Cl, ldC, PC, G, Dl, Dh, Dlo, ldD, lam_in,
                                        eta, st, pu));
          } else if (f32_steps) {
            LR_HIP(lr::step_dot_f32(X, p, b, it, scale + (t - t0) * b, D32, C32, PC, st, pd));
            LR_HIP(lr::step_update_f32(X, p, b, it, C32, PC, G, Dl, D32, lam_in, eta, st, pu));
          } else {
            LR_HIP(lr::step_dot(X, pc, b, it, scale + (t - t0) * b, Dl, C, PCn, st, pd));
            LR_HIP(lr::step_update(X, pc, b, it, C, PCn, G, Dl, lam_in, eta, st, pu, df));
          }
        }
      }
      if (sparse) LR_HIP(lr::rm_to_cm(Dlrm, d, p, PC, Dl, st));
      if (opt.timing) LR_HIP(hipEventRecord(ev[1], st));
      rep.steps += m;
      if (accel) {
        // W_k = W_{k-1} + Delta; G = (lam + kappa) W_k - A W_k - (S + kappa Y_{k-1})
        if (tiled)
          LR_HIP(lr::tile_add(d, pc, PCn, Wt, Dl, Wn, st));
        else
          LR_HIP(lr::lincomb(cnt, 1.0, Wt, 1.0, Dl, 0.0, nullptr, Wn, st));
        LR_HIP(lr::lincomb(cnt, 1.0, Srhs, kappa, Yk, 0.0, nullptr, Racc, st));
        if (opt.timing) LR_HIP(hipEventRecord(ev[2], st));
        LR_CHECK(applyA(Wn, G, pc, -1.0, Wn, lam_in, Racc, -1.0));
        if (opt.timing) LR_HIP(hipEventRecord(ev[3], st));
        // residual of the original system: kappa (W_k - Y_{k-1}) - G
        LR_HIP(lr::lincomb(cnt, kappa, Wn, -kappa, Yk, -1.0, G, Tm1, st));
        LR_HIP(lr::sumsq(Tm1, cnt, part, dnorm, st));
        // Y_k = W_k + beta (W_k - W_{k-1}); the next gradient G - kappa (Y_k - Y_{k-1})
        LR_HIP(lr::lincomb(cnt, 1.0 + beta, Wn, -beta, Wt, 0.0, nullptr, Ynew, st));
        LR_HIP(lr::lincomb(cnt, 1.0, G, -kappa, Ynew, kappa, Yk, G, st));
        std::swap(Yk, Ynew);
        std::swap(Wt, Wn);
      } else if (mc) {
        // residual refinement: G~ is linear in W~, so the new anchor's gradient is
        // the old one plus lam D - X X^T D for the epoch's difference D = W~' - W~;
        // the matrix-core pass then errs relative to D rather than to W~
        if (tiled)
          LR_HIP(lr::tile_add(d, pc, PCn, Wt, Dl, Tm1, st));
        else
          LR_HIP(lr::lincomb(cnt, 1.0, Wt, 1.0, Dl, 0.0, nullptr, Tm1, st));
        LR_HIP(lr::lincomb(cnt, 1.0, Tm1, -1.0, Wt, 0.0, nullptr, Tm2, st));
        if (opt.timing) LR_HIP(hipEventRecord(ev[2], st));
        LR_CHECK(applyA(Tm2, G, pc, -1.0, Tm2, lam, G, 1.0));
        if (opt.timing) LR_HIP(hipEventRecord(ev[3], st));
        LR_HIP(hipMemcpyAsync(Wt, Tm1, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
        LR_HIP(lr::sumsq(G, cnt, part, dnorm, st));
      } else {
        if (tiled)
          LR_HIP(lr::tile_add(d, pc, PCn, Wt, Dl, Wt, st));
        else
          LR_HIP(lr::lincomb(cnt, 1.0, Wt, 1.0, Dl, 0.0, nullptr, Wt, st));
        if (opt.timing) LR_HIP(hipEventRecord(ev[2], st));
        LR_CHECK(applyA(Wt, G, pc, -1.0, Wt, lam, Srhs, -1.0));
        if (opt.timing) LR_HIP(hipEventRecord(ev[3], st));
        LR_HIP(lr::sumsq(G, cnt, part, dnorm, st));
      }
      LR_CHECK(read(&r, dnorm, sizeof(double)));
      r = std::sqrt(r);
      if (opt.timing) {
        float ms = 0;
        LR_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        rep.ms_steps_total += ms;
        rep.timed_steps += m;
        LR_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
        rep.ms_pass_total += ms;
        rep.timed_passes += 1;
        LR_HIP(hipEventElapsedTime(&ms, ev[4], ev[5]));
        rep.ms_sample_dot_probe += ms;
        LR_HIP(hipEventElapsedTime(&ms, ev[6], ev[7]));
        rep.ms_update_probe += ms;
        rep.probes += 1;
      }
      ++e;
      if (hist) hist->push_back(r);
      if (!std::isfinite(r) || r > 1e3 * r0)
        return fail(LR_ESHIFT, "inner solver diverged: shift not above lambda_1");
    }
    rep.total_epochs += e;
    if (epochs_out) *epochs_out = e;
    return LR_OK;
  }

  lr_status estimate(int pc, int interval, double* theta, double* resn);
  // The rough upper bound mu on ||X|| / ||X - X_k|| by which eps is rescaled
  // (Corollary "mainResult"), from the estimate-phase Ritz values: Frobenius
  // ||X||_F / sqrt(||X||_F^2 - sum_{i<=k} theta_i), spectral sqrt(theta_1 / theta_{k+1}).
  double stop_scale(const double* theta) const {
    if (opt.norm == 1) return std::sqrt(theta[0] / std::max(theta[k], 1e-300));
    double top = 0;
    for (int i = 0; i < k; ++i) top += theta[i];
    return std::sqrt(fro2 / std::max(fro2 - top, 1e-300));
  }
  lr_status tune_shift(const double* theta, const double* resn, double delta, int pc,
                       int32_t solve0, bool record, double* lam_out, double* mu_out,
                       int* rounds_out, double* nu_out);
  lr_status subspace_change(const double* A, const double* B, int cols, double* change);
  lr_status power_deflated(int cols, int interval, double eps_stop, int* iters, bool* ok);
  lr_status si_deflated(double lam, double eta, int64_t m, int64_t b, double tau,
                        double eps_stop, int32_t first_solve, int target, int cols, int* outer,
                        bool* ok, double kappa = 0.0, double beta = 0.0);
  lr_status append_basis(const double* B, int cols);
  lr_status final_rr(const double* Sb, int cols, double* U_out, double* theta_out);
  lr_status solve(double* U_out, double* theta_out, lr_report* out_rep);
  lr_status solve_adaptive(double* U_out, double* theta_out, lr_report* out_rep);
  lr_status solve_intervals();
};

// Algorithm "musco" on the (deflated) A with a block of pc columns (random start
// of stream (tag 1, interval)): est_iters plain steps, Rayleigh-Ritz, residual
// norms.  The block is left in Sest; theta, resn: host, pc values.
lr_status lr_plan_s::estimate(int pc, int interval, double* theta, double* resn) {
  LR_HIP(lr::gaussian(Sest, d, pc, opt.seed, stream_word(TAG_EST_INIT, (uint32_t)interval), st));
  if (ns > 0) LR_CHECK(deflate(Sest, Sest, pc));
  LR_CHECK(cholqr2(Sest, Sest, pc));
  for (int it = 0; it < opt.est_iters; ++it) {
    LR_CHECK(applyA(Sest, Y, pc));
    LR_CHECK(cholqr2(Y, Sest, pc));
  }
  LR_CHECK(applyA(Sest, Y, pc));
  LR_CHECK(gram_dd(Sest, pc, Y, pc, H));
  LR_HIP(lr::eigh(H, pc, vals, Q, st));
  LR_HIP(lr::gemm_small(d, pc, pc, Y, Q, pc, Tm1, 0.0, nullptr, st));
  LR_HIP(lr::gemm_small(d, pc, pc, Sest, Q, pc, Tm2, 0.0, nullptr, st));
  LR_HIP(lr::residual_norms(Tm1, Tm2, vals, d, pc, res, st));
  LR_CHECK(check_spd());
  LR_CHECK(read(theta, vals, pc * sizeof(double)));
  LR_CHECK(read(resn, res, pc * sizeof(double)));
  return LR_OK;
}

// Algorithm shiftTune on the estimate block Sest (pc columns): aim
// 1/nu_1 ~ lambda - lambda_1 into [Delta/27, Delta/5].  Inner solves use solve
// indices solve0, solve0 + 1, ...  nu_out (may be null): the pc Ritz values of
// the last round.
lr_status lr_plan_s::tune_shift(const double* theta, const double* resn, double delta, int pc,
                                int32_t solve0, bool record, double* lam_out, double* mu_out,
                                int* rounds_out, double* nu_out) {
  const double t1 = theta[0], r1 = resn[0];
  double lam, mu;
  if (opt.shift_start > 0) {
    lam = opt.shift_start;
    mu = std::max(lam - t1 - r1, delta / 30.0);
  } else if (opt.shift_mode == 1) {
    lam = 1.5 * t1;
    mu = std::max(lam - t1 - r1, delta / 30.0);
  } else {
    lam = t1 + r1 + delta / 10.0;
    mu = delta / 10.0;
  }
  for (int r = 0; r < opt.max_shift_rounds; ++r) {
    const Inner ic = inner_constants(t1, lam, mu);
    LR_CHECK(svrg_solve(Sest, lam, ic.eta, ic.m, ic.b, solve0 + r, opt.tau_shift, -1, nullptr,
                        nullptr, pc, ic.kappa, ic.beta));
    LR_CHECK(gram_dd(Sest, pc, Wt, pc, H));
    LR_HIP(lr::eigh(H, pc, vals, Q, st));
    double nu[LR_MAX_P];
    LR_CHECK(read(nu, vals, pc * sizeof(double)));
    if (nu_out) std::memcpy(nu_out, nu, pc * sizeof(double));
    const double nu1 = nu[0];
    if (!(nu1 > 0)) return fail(LR_ESHIFT, "shift estimate not positive");
    const double g = 1.0 / nu1;
    if (record && r < LR_MAX_SHIFT_ROUNDS) {
      rep.shift_lambda[r] = lam;
      rep.shift_gap[r] = g;
    }
    *rounds_out = r + 1;
    if (delta / 27.0 <= g && g <= delta / 5.0) {
      *lam_out = lam;
      *mu_out = g;
      return LR_OK;
    }
    if (g > delta / 5.0) {
      lam -= (4.0 / 9.0) * g;
      mu = (5.0 / 9.0) * g;
    } else {
      lam += delta / 10.0;
      mu = g + delta / 10.0;
    }
  }
  return fail(LR_ESHIFT, "shift tuning did not reach the target interval");
}

lr_status lr_plan_s::solve(double* U_out, double* theta_out, lr_report* out_rep) {
  rep = lr_report{};
  epochs.clear();
  LR_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), st));
  LR_CHECK(prepare());
  rep.fro2 = fro2;
  sched = lr_schedule{};
  const int64_t cnt = d * p;
  double theta[LR_MAX_P], resn[LR_MAX_P];
  if (!replay) {
    // estimate phase: subspace iteration on A with p columns, then Rayleigh-Ritz
    LR_CHECK(estimate(p, 0, theta, resn));
    for (int i = 0; i < p; ++i) {
      rep.theta_est[i] = theta[i];
      rep.res_est[i] = resn[i];
    }
    const double delta = (theta[k - 1] - theta[p - 1]) / 1.5;
    if (!(delta > 1e-12 * theta[0])) return fail(LR_ENOGAP, "no gap between theta_k and theta_p");
    const double muF = stop_scale(theta);
    rep.mu_F = muF;
    const double eps_stop = eps / (k * muF);
    const double tau = std::min(1e-2, 0.1 * eps_stop);
    const double t1 = theta[0];
    double lam = 0, mu = 0;
    int rounds = 0;
    LR_CHECK(tune_shift(theta, resn, delta, p, 0, true, &lam, &mu, &rounds, nullptr));
    rep.shift_rounds = rounds;
    sched.lambda = lam;
    sched.mu_hat = mu;
    sched.delta_hat = delta;
    const Inner ic = inner_constants(t1, lam, mu);
    sched.b = ic.b;
    sched.eta = ic.eta;
    sched.m = ic.m;
    acc_kappa = ic.kappa;
    acc_beta = ic.beta;
    rep.accel_kappa = ic.kappa;
    rep.accel_beta = ic.beta;
    sched.tau = tau;
    sched.eps_stop = eps_stop;
    sched.first_solve = rounds;
  } else {
    sched = rsched;
    sched.epochs = nullptr;
    sched.n_epochs = 0;
  }
  // shift-and-invert subspace iteration, p' = p
  LR_HIP(lr::gaussian(S, d, p, opt.seed, stream_word(TAG_SI_INIT, (uint32_t)sched.first_solve),
                      st));
  LR_CHECK(cholqr2(S, S, p));
  const int L = replay ? rsched.outer : opt.max_outer;
  bool converged = replay;
  double change = -1.0;
  for (int ell = 0; ell < L; ++ell) {
    int32_t e = 0;
    mc_active = mc_pass;
    const lr_status si = svrg_solve(S, sched.lambda, sched.eta, sched.m, sched.b,
                                    sched.first_solve + ell, sched.tau,
                                    replay ? repochs[ell] : -1, &e, nullptr, -1, acc_kappa,
                                    acc_beta);
    mc_active = false;
    LR_CHECK(si);
    epochs.push_back(e);
    LR_CHECK(gram_dd(S, p, Wt, p, H));
    LR_HIP(lr::eigh(H, p, vals, Q, st));
    LR_HIP(lr::gemm_small(d, p, k, S, Q, p, V, 0.0, nullptr, st));
    LR_CHECK(cholqr2(Wt, S, p));
    if (ell > 0) {
      LR_HIP(lr::gram(Vprev, 1, d, k, V, 1, d, k, d, part, kk1, st));
      LR_HIP(lr::gram(kk1, 1, k, k, kk1, 1, k, k, k, part, kk2, st));
      LR_HIP(lr::eigh(kk2, k, vals, Q, st));
      double lmin;
      LR_CHECK(read(&lmin, vals + (k - 1), sizeof(double)));
      change = std::sqrt(std::max(0.0, 1.0 - lmin));
      if (!replay && change <= sched.eps_stop) {
        converged = true;
        break;
      }
    }
    std::swap(V, Vprev);
  }
  LR_CHECK(check_spd());
  sched.outer = (int32_t)epochs.size();
  rep.outer = sched.outer;
  rep.last_change = change;
  // final Rayleigh-Ritz with C = XX^T: H = (X^T S)^T (X^T S), one half pass
  for (int it = 0; it < opt.polish; ++it) {
    LR_CHECK(applyA(S, Y, p));
    LR_CHECK(cholqr2(Y, S, p));
  }
  LR_CHECK(xtw(S, p));
  LR_HIP(lr::gram(T, PC, 1, p, T, PC, 1, p, n, part, H, st));
  LR_HIP(lr::eigh(H, p, vals, Q, st));
  double* Uo = U_out ? U_out : Tm2;
  LR_HIP(lr::gemm_small(d, p, k, S, Q, p, Uo, 0.0, nullptr, st));
  LR_HIP(lr::sign_fix(Uo, d, k, st));
  double th[LR_MAX_P];
  LR_CHECK(read(th, vals, k * sizeof(double)));
  LR_CHECK(check_spd());
  if (theta_out) std::memcpy(theta_out, th, k * sizeof(double));
  (void)cnt;
  if (out_rep) *out_rep = rep;
  if (!converged) return fail(LR_ENOCONV, "outer iteration reached max_outer");
  return LR_OK;
}

// sin of the largest principal angle between span(A) and span(B) (d x cols,
// orthonormal): sqrt(1 - lambda_min((A^T B)^T (A^T B))).
lr_status lr_plan_s::subspace_change(const double* A, const double* B, int cols, double* change) {
  LR_HIP(lr::gram(A, 1, d, cols, B, 1, d, cols, d, part, kk1, st));
  LR_HIP(lr::gram(kk1, 1, cols, cols, kk1, 1, cols, cols, cols, part, kk2, st));
  LR_HIP(lr::eigh(kk2, cols, vals, Q, st));
  double lmin;
  LR_CHECK(read(&lmin, vals + (cols - 1), sizeof(double)));
  *change = std::sqrt(std::max(0.0, 1.0 - lmin));
  return LR_OK;
}

// Plain subspace iteration on the deflated A with `cols` columns and no
// oversampling (the largeDetect branch of Algorithm "main"); the block is left
// in S.  Stops when its span moves by at most eps_stop.
lr_status lr_plan_s::power_deflated(int cols, int interval, double eps_stop, int* iters,
                                    bool* ok) {
  LR_HIP(lr::gaussian(S, d, cols, opt.seed, stream_word(TAG_POWER_INIT, (uint32_t)interval), st));
  if (ns > 0) LR_CHECK(deflate(S, S, cols));
  LR_CHECK(cholqr2(S, S, cols));
  *ok = false;
  int it = 0;
  while (it < opt.max_outer) {
    LR_CHECK(applyA(S, Y, cols));
    LR_CHECK(cholqr2(Y, W, cols));
    double ch;
    LR_CHECK(subspace_change(S, W, cols, &ch));
    std::swap(S, W);
    ++it;
    if (ch <= eps_stop) {
      *ok = true;
      break;
    }
  }
  *iters = it;
  return LR_OK;
}

// Shift-and-invert subspace iteration on the deflated operator with `cols`
// columns; stops when the top-`target` Ritz subspace moves by at most
// eps_stop.  The block is left in S.
lr_status lr_plan_s::si_deflated(double lam, double eta, int64_t m, int64_t b, double tau,
                                 double eps_stop, int32_t first_solve, int target, int cols,
                                 int* outer, bool* ok, double kappa, double beta) {
  LR_HIP(lr::gaussian(S, d, cols, opt.seed, stream_word(TAG_SI_INIT, (uint32_t)first_solve), st));
  if (ns > 0) LR_CHECK(deflate(S, S, cols));
  LR_CHECK(cholqr2(S, S, cols));
  *ok = false;
  int ell = 0;
  while (ell < opt.max_outer) {
    int32_t e = 0;
    LR_CHECK(svrg_solve(S, lam, eta, m, b, first_solve + ell, tau, -1, &e, nullptr, cols, kappa,
                        beta));
    epochs.push_back(e);
    LR_CHECK(gram_dd(S, cols, Wt, cols, H));
    LR_HIP(lr::eigh(H, cols, vals, Q, st));
    LR_HIP(lr::gemm_small(d, cols, target, S, Q, cols, V, 0.0, nullptr, st));
    LR_CHECK(cholqr2(Wt, S, cols));
    ++ell;
    if (ell > 1) {
      double ch;
      LR_CHECK(subspace_change(Vprev, V, target, &ch));
      rep.last_change = ch;
      if (ch <= eps_stop) {
        *ok = true;
        break;
      }
    }
    std::swap(V, Vprev);
  }
  *outer = ell;
  return LR_OK;
}

// Append B (d x cols) to the deflation basis: Ud[:, ns:ns+cols] = CholQR2(P B);
// then Z = X^T Ud for the deflated inner steps.
lr_status lr_plan_s::append_basis(const double* B, int cols) {
  if (ns + cols > p) return fail(LR_EINVAL, "deflation basis full");
  if (ns > 0)
    LR_CHECK(deflate(B, Tm2, cols));
  else
    LR_HIP(hipMemcpyAsync(Tm2, B, d * cols * sizeof(double), hipMemcpyDeviceToDevice, st));
  LR_CHECK(cholqr2(Tm2, Ud + (int64_t)ns * d, cols));
  ns += cols;
  LR_HIP(lr::pass_xtw(X, Ud, ns, Zt, lr::pad16(ns), Wtl, st));
  return LR_OK;
}

// Algorithm "second stage" with C = XX^T on the orthonormal block Sb (cols
// columns): H = (X^T Sb)^T (X^T Sb), U_k = Sb Q[:, :k], theta = top k of eig H.
lr_status lr_plan_s::final_rr(const double* Sb, int cols, double* U_out, double* theta_out) {
  LR_CHECK(xtw(Sb, cols));
  LR_HIP(lr::gram(T, PC, 1, cols, T, PC, 1, cols, n, part, H, st));
  LR_HIP(lr::eigh(H, cols, vals, Q, st));
  double* Uo = U_out ? U_out : Tm2;
  LR_HIP(lr::gemm_small(d, cols, k, Sb, Q, cols, Uo, 0.0, nullptr, st));
  LR_HIP(lr::sign_fix(Uo, d, k, st));
  double th[LR_MAX_P];
  LR_CHECK(read(th, vals, k * sizeof(double)));
  LR_CHECK(check_spd());
  if (theta_out) std::memcpy(theta_out, th, k * sizeof(double));
  return LR_OK;
}

// Algorithm "main" with adaptive partitioning (Section 3.2): intervals s..q
// taken by plain subspace iteration on the deflated A when largeDetect finds a
// multiplicative gap, else by shift-and-invert iteration on the deflated
// operator, split where deltaDetect finds an additive gap.
//
// Readings: largeDetect returns the largest qualifying q; the estimates of
// Algorithm "musco" on the deflated inverse are the Ritz values of the last
// shiftTune round; the gap budget and the stopping threshold come from the
// first interval; deflated columns are sampled with the undeflated weights.
lr_status lr_plan_s::solve_adaptive(double* U_out, double* theta_out, lr_report* out_rep) {
  rep = lr_report{};
  epochs.clear();
  sched = lr_schedule{};
  ns = 0;
  LR_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), st));
  LR_CHECK(prepare());
  rep.fro2 = fro2;
  lr_status res_ = solve_intervals();
  const int nb = ns;
  ns = 0;   // the final Rayleigh-Ritz and later calls see the undeflated A
  LR_CHECK(res_ == LR_ENOCONV ? LR_OK : res_);
  LR_CHECK(final_rr(Ud, nb, U_out, theta_out));
  if (out_rep) *out_rep = rep;
  if (res_ == LR_ENOCONV) return fail(LR_ENOCONV, "an iteration reached max_outer");
  return LR_OK;
}

lr_status lr_plan_s::solve_intervals() {
  int s0 = 0, t = 0;
  int32_t solve_ctr = 0;
  double delta = 0, eps_stop = 0, tau = 0;
  bool all_ok = true;
  while (s0 < k) {
    const int kk = k - s0, pc = p - s0;
    double theta[LR_MAX_P], resn[LR_MAX_P];
    LR_CHECK(estimate(pc, t, theta, resn));
    if (t == 0) {
      for (int i = 0; i < p; ++i) {
        rep.theta_est[i] = theta[i];
        rep.res_est[i] = resn[i];
      }
      delta = (theta[k - 1] - theta[p - 1]) / 1.5;
      if (!(delta > 1e-12 * theta[0])) return fail(LR_ENOGAP, "no gap between theta_k and theta_p");
      const double muF = stop_scale(theta);
      rep.mu_F = muF;
      eps_stop = eps / (k * muF);
      tau = std::min(1e-2, 0.1 * eps_stop);
      sched.delta_hat = delta;
      sched.eps_stop = eps_stop;
      sched.tau = tau;
    }
    // Algorithm largeDetect: the largest q in I \ {k} with a multiplicative gap
    int q = -1;
    for (int i = 0; i + 1 < kk; ++i)
      if (theta[i + 1] <= theta[i] * (1.0 - 1.0 / ((double)p * p))) q = i;
    int cols = 0, iters = 0, branch = 0;
    bool ok = false;
    if (q >= 0) {
      cols = q + 1;
      LR_CHECK(power_deflated(cols, t, eps_stop, &iters, &ok));
      LR_CHECK(append_basis(S, cols));
    } else {
      branch = 1;
      double lam = 0, mu = 0, nu[LR_MAX_P];
      int rounds = 0;
      LR_CHECK(tune_shift(theta, resn, delta, pc, solve_ctr, t == 0, &lam, &mu, &rounds, nu));
      if (t == 0) rep.shift_rounds = rounds;
      solve_ctr += rounds;
      // Algorithm deltaDetect on the estimates 1/nu_i of lambda - lambda_i
      q = kk - 1;
      for (int i = 0; i + 1 < kk; ++i)
        if (1.0 / nu[i + 1] - 1.0 / nu[i] >= 5.0 * delta / 9.0) {
          q = i;
          break;
        }
      cols = q == kk - 1 ? pc : q + 1;
      const Inner ic = inner_constants(theta[0], lam, mu);
      sched.lambda = lam;
      sched.mu_hat = mu;
      sched.eta = ic.eta;
      sched.m = ic.m;
      sched.b = ic.b;
      rep.accel_kappa = ic.kappa;
      rep.accel_beta = ic.beta;
      LR_CHECK(si_deflated(lam, ic.eta, ic.m, ic.b, tau, eps_stop, solve_ctr, q + 1, cols, &iters,
                           &ok, ic.kappa, ic.beta));
      solve_ctr += iters;
      if (q < kk - 1) {   // keep the interval's own directions: top Ritz vectors in span(S)
        LR_CHECK(applyA(S, Y, cols));
        LR_CHECK(gram_dd(S, cols, Y, cols, H));
        LR_HIP(lr::eigh(H, cols, vals, Q, st));
        LR_HIP(lr::gemm_small(d, cols, q + 1, S, Q, cols, Tm1, 0.0, nullptr, st));
        LR_CHECK(append_basis(Tm1, q + 1));
      } else {
        LR_CHECK(append_basis(S, cols));
      }
    }
    if (t < LR_MAX_P) {
      rep.interval_s[t] = s0 + 1;
      rep.interval_q[t] = s0 + q + 1;
      rep.interval_branch[t] = branch;
      rep.interval_cols[t] = cols;
      rep.interval_iters[t] = iters;
    }
    all_ok = all_ok && ok;
    s0 += q + 1;
    ++t;
  }
  rep.n_intervals = t;
  rep.outer = (int32_t)epochs.size();
  sched.outer = rep.outer;
  return all_ok ? LR_OK : LR_ENOCONV;
}

size_t lr_plan_s::carve(char* base) {
  size_t off = 0;
  auto take = [&](auto** ptr, int64_t count) {
    off = (off + 255) & ~(size_t)255;
    if (base) *ptr = reinterpret_cast<std::remove_pointer_t<decltype(ptr)>>(base + off);
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(**ptr);
  };
  const int64_t dp = d * p;
  const int64_t nbt = (n + 1023) / 1024;
  const int64_t partn = std::max<int64_t>((int64_t)lr::gram_nblk(std::max(d, n)) * 64 * 64, 1024);
  take(&w, n);
  take(&cdf, n + 1);
  take(&scratch, 3 * nbt + 8);
  for (double** b : {&S, &W, &Wt, &G, &Y, &Tm1, &Tm2, &Sest}) take(b, dp);
  take(&Dl, std::max<int64_t>(dp, lr::pad16(d) * PC));   // tile-major on the dense FP64 path
  take(&Wtl, sparse ? 0 : lr::pad16(d) * PC);             // tile-major W for the dense pass
  take(&V, d * k);
  take(&Vprev, d * k);
  for (double** b : {&Wrm, &Grm, &Dlrm}) take(b, sparse ? d * PC : 0);
  for (uint16_t** b : {&Dh, &Dlo}) take(b, bf16_steps ? ldD * PC : 0);
  for (double** b : {&Ud, &Dw1, &Dw2}) take(b, adaptive ? d * p : 0);
  for (double** b : {&Wn, &Ya, &Yb, &Racc}) take(b, accel ? d * p : 0);
  take(&Zt, adaptive ? n * PC : 0);
  take(&Kd, adaptive ? 64 * 64 : 0);
  take(&Vp, adaptive ? (int64_t)lr::zbc_chunks(bmax) * 64 * 64 : 0);
  for (uint16_t** b : {&Ch, &Cl}) take(b, bf16_steps ? ldC * PC : 0);
  take(&D32, f32_steps ? lr::pad16(d) * PC : 0);
  {
    const lr::McSizes z = mc_pass ? lr::mc_sizes(d, n, PC) : lr::McSizes{0, 0, 0, 0};
    take(&mb.Wp, z.wp_elems);
    take(&mb.Tp, z.tp_elems);
    take(&mb.part, z.part_elems);
    mb.wstride = z.wp_elems / 3;
    mb.tstride = z.tp_elems / 3;
    mb.nsplit = z.nsplit;
  }
  take(&C32, f32_steps ? 2 * lr::pad16(bmax) * PC : 0);   // two row-split partials
  take(&T, n * PC);
  take(&Ypart, (int64_t)pb.nsplit * dp);
  take(&C, lr::pad16(bmax) * PC);   // zero rows past b up to a multiple of 16
  take(&scale, MCH * bmax);
  take(&idx, MCH * bmax);
  take(&part, partn);
  for (double** b : {&H, &Q, &M, &Rinv, &kk1, &kk2}) take(b, 64 * 64);
  take(&vals, 64);
  take(&res, 64);
  take(&dfro2, 1);
  take(&dnorm, 4);
  take(&dinfo, 1);
  take(&dbad, 1);
  if (base) pb.Ypart = Ypart;
  return (off + 255) & ~(size_t)255;
}

// Device structure checks of the caller's CSC arrays: *bad = 0 when sound, 1
// when col_ptr does not rise from 0 to nnz, 2 when a row id is out of [0, d) or
// not increasing within its column.
lr_status lr_plan_s::device_structure(int* bad) {
  *bad = 0;
  LR_HIP(hipMemsetAsync(dbad, 0, sizeof(int), st));
  LR_HIP(lr::csc_check_ptr(Xs, dbad, st));
  LR_CHECK(read(bad, dbad, sizeof(int)));
  if (*bad) return LR_OK;
  LR_HIP(lr::csc_check_rows(Xs, dbad, st));
  LR_CHECK(read(bad, dbad, sizeof(int)));
  return LR_OK;
}

namespace {
// The same structure rules on host copies; "" when sound, else the first
// violation.
std::string host_structure(const std::vector<int32_t>& cp, const std::vector<int32_t>& ri,
                           int64_t n, int64_t nnz, int64_t d) {
  char buf[160];
  if (cp[0] != 0 || cp[n] != nnz) {
    std::snprintf(buf, sizeof buf, "CSC col_ptr must rise from 0 to nnz (col_ptr[0] = %d, "
                  "col_ptr[n] = %d, nnz = %lld)", cp[0], cp[n], (long long)nnz);
    return buf;
  }
  for (int64_t i = 0; i < n; ++i)
    if (cp[i + 1] < cp[i] || cp[i] < 0 || cp[i] > nnz) {
      std::snprintf(buf, sizeof buf, "CSC col_ptr must rise from 0 to nnz (col_ptr[%lld] = %d, "
                    "col_ptr[%lld] = %d)", (long long)i, cp[i], (long long)(i + 1), cp[i + 1]);
      return buf;
    }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = cp[i]; k < cp[i + 1]; ++k)
      if (ri[k] < 0 || ri[k] >= d || (k > cp[i] && ri[k] <= ri[k - 1])) {
        std::snprintf(buf, sizeof buf, "CSC row ids must lie in [0, d) and increase within each "
                      "column (column %lld, entry %lld: row %d)", (long long)i, (long long)k,
                      ri[k]);
        return buf;
      }
  return "";
}
}  // namespace

// A device check rejected X: copy col_ptr and row_idx to the host and apply the
// same rules there.  If the host copy breaks them, LR_EINVAL names the first
// violation.  If it does not, the device check read something other than what
// the arrays hold; it is run once more, and a second rejection is LR_EDEVICE
// (the input is not blamed for what the device saw).
lr_status lr_plan_s::confirm_structure(int device_flag) {
  const int64_t n = Xs.n, nnz = Xs.nnz;
  std::vector<int32_t> cp(n + 1), ri(std::max<int64_t>(nnz, 1));
  LR_HIP(hipStreamSynchronize(st));
  LR_HIP(hipMemcpy(cp.data(), Xs.cp, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  const bool ptr_ok = cp[0] == 0 && cp[n] == nnz &&
                      [&] {
                        for (int64_t i = 0; i < n; ++i)
                          if (cp[i + 1] < cp[i] || cp[i] < 0) return false;
                        return true;
                      }();
  if (ptr_ok && nnz > 0)
    LR_HIP(hipMemcpy(ri.data(), Xs.ri, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  const std::string why = host_structure(cp, ri, n, nnz, d);
  if (!why.empty()) return fail(LR_EINVAL, why);
  int again = 0;
  LR_CHECK(device_structure(&again));
  if (again) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "device check of the CSC structure flagged %d then %d, but a "
                  "host copy of col_ptr and row_idx is sound", device_flag, again);
    return fail(LR_EDEVICE, buf);
  }
  return LR_OK;
}

lr_status lr_plan_s::sparse_setup() {
  const int64_t nnz = Xs.nnz;
  const size_t elt = Xs.dt == LR_F64 ? 8 : Xs.dt == LR_F32 ? 4 : 2;
  auto keep = [&](void** ptr, size_t bytes) -> lr_status {
    if (hipMalloc(ptr, std::max<size_t>(bytes, 1)) != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      return fail(LR_ENOMEM, "device allocation failed");
    }
    sp_allocs.push_back(*ptr);
    if (opt.fill_workspace && lr::fill_bytes(*ptr, std::max<size_t>(bytes, 1) & ~(size_t)3, 0xFF,
                                             st) != hipSuccess)
      return fail(LR_EDEVICE, "workspace fill failed");
    return LR_OK;
  };
  // structure checks on the device; row ids are read only once col_ptr is
  // known to be sound.  A rejection is confirmed on a host copy of the arrays
  // before it is reported (see confirm_structure).
  int bad = 0;
  LR_CHECK(device_structure(&bad));
  if (bad) LR_CHECK(confirm_structure(bad));
  // row-ordered copy: stable radix sort of the row ids keeps columns ascending
  void *col = nullptr, *val = nullptr;
  LR_CHECK(keep(&col, (size_t)nnz * 4));
  LR_CHECK(keep(&val, (size_t)nnz * elt));
  size_t tb = 0;
  LR_HIP(lr::csr_sort_bytes(nnz, d, &tb));
  void* tmp[5] = {};
  const size_t tmp_bytes[5] = {tb, (size_t)nnz * 4, (size_t)nnz * 4, (size_t)nnz * 4,
                               (size_t)(d + 1) * 4};
  lr_status s = LR_OK;
  for (int i = 0; i < 5 && s == LR_OK; ++i)
    if (hipMalloc(&tmp[i], std::max<size_t>(tmp_bytes[i], 1)) != hipSuccess) {
      (void)hipGetLastError();
      tmp[i] = nullptr;
      s = fail(LR_ENOMEM, "device allocation failed");
    }
  std::vector<int32_t> row_ptr(d + 1);
  if (s == LR_OK) {
    hipError_t e = lr::csr_build(Xs, tmp[0], tb, (uint32_t*)tmp[1], (int32_t*)tmp[2],
                                 (int32_t*)tmp[3], (int32_t*)tmp[4], (int32_t*)col, val, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(row_ptr.data(), tmp[4], (d + 1) * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = fail(LR_EDEVICE, std::string("CSR build: ") + hipGetErrorString(e));
  }
  (void)hipStreamSynchronize(st);
  for (void* t : tmp)
    if (t) (void)hipFree(t);
  LR_CHECK(s);
  // chunks of at most SP_CHUNK entries per row; rows without entries own none
  std::vector<int32_t> row_chunk(d + 1), chunk_beg;
  chunk_beg.reserve(d + nnz / lr::SP_CHUNK + 2);
  for (int64_t r = 0; r < d; ++r) {
    row_chunk[r] = (int32_t)chunk_beg.size();
    for (int64_t b = row_ptr[r]; b < row_ptr[r + 1]; b += lr::SP_CHUNK) chunk_beg.push_back((int32_t)b);
  }
  row_chunk[d] = (int32_t)chunk_beg.size();
  const int64_t nch = (int64_t)chunk_beg.size();
  chunk_beg.push_back((int32_t)nnz);
  // head rows: the rows stored most often, summed per workgroup in LDS by the
  // inner-step scatter
  std::vector<int32_t> order(d);
  for (int64_t r = 0; r < d; ++r) order[r] = (int32_t)r;
  const int64_t hcap = std::min<int64_t>(d, lr::sp_head_cap(PC));
  std::partial_sort(order.begin(), order.begin() + hcap, order.end(), [&](int32_t a, int32_t b) {
    const int32_t ca = row_ptr[a + 1] - row_ptr[a], cb = row_ptr[b + 1] - row_ptr[b];
    return ca != cb ? ca > cb : a < b;
  });
  int H = 0;
  while (H < hcap && row_ptr[order[H] + 1] > row_ptr[order[H]]) ++H;
  std::vector<int32_t> head_slot(d, -1), head_row(std::max(H, 1), 0);
  for (int h = 0; h < H; ++h) {
    head_slot[order[h]] = h;
    head_row[h] = order[h];
  }
  void *rc = nullptr, *cb = nullptr, *hs = nullptr, *hr = nullptr, *pt = nullptr;
  LR_CHECK(keep(&rc, row_chunk.size() * 4));
  LR_CHECK(keep(&cb, chunk_beg.size() * 4));
  LR_CHECK(keep(&hs, head_slot.size() * 4));
  LR_CHECK(keep(&hr, head_row.size() * 4));
  LR_CHECK(keep(&pt, (size_t)std::max<int64_t>(nch, 1) * PC * 8));
  LR_HIP(hipMemcpyAsync(rc, row_chunk.data(), row_chunk.size() * 4, hipMemcpyHostToDevice, st));
  LR_HIP(hipMemcpyAsync(cb, chunk_beg.data(), chunk_beg.size() * 4, hipMemcpyHostToDevice, st));
  LR_HIP(hipMemcpyAsync(hs, head_slot.data(), head_slot.size() * 4, hipMemcpyHostToDevice, st));
  LR_HIP(hipMemcpyAsync(hr, head_row.data(), head_row.size() * 4, hipMemcpyHostToDevice, st));
  LR_HIP(hipStreamSynchronize(st));
  R = lr::CsrView{(const int32_t*)col, val, (const int32_t*)cb, (const int32_t*)rc, d, nch,
                  Xs.dt};
  sp_head_slot = (int32_t*)hs;
  sp_head_row = (int32_t*)hr;
  sp_H = H;
  sp_part = (double*)pt;
  // the inner step's scatter in a fixed order needs room for bmax x (most
  // entries in a column) contributions; past the cap it stays with atomics
  std::vector<int32_t> cph(Xs.n + 1);
  LR_HIP(hipMemcpyAsync(cph.data(), Xs.cp, (Xs.n + 1) * 4, hipMemcpyDeviceToHost, st));
  LR_HIP(hipStreamSynchronize(st));
  int64_t maxnnz = 0;
  for (int64_t i = 0; i < Xs.n; ++i) maxnnz = std::max<int64_t>(maxnnz, cph[i + 1] - cph[i]);
  const int64_t tmax = bmax * maxnnz;
  if (maxnnz >= 1 && tmax <= lr::SP_SORT_CAP) {
    // the same buffers as lr::sp_sort_bytes counts for plan_bytes
    void *ki = nullptr, *ko = nullptr, *pi = nullptr, *po = nullptr, *xv = nullptr,
         *hs2 = nullptr, *ca = nullptr, *fl = nullptr;
    const int64_t nchs = lr::sp_chunks(tmax);
    LR_CHECK(keep(&ki, (size_t)tmax * 4));
    LR_CHECK(keep(&ko, (size_t)tmax * 4));
    LR_CHECK(keep(&pi, (size_t)tmax * 4));
    LR_CHECK(keep(&po, (size_t)tmax * 4));
    LR_CHECK(keep(&xv, (size_t)tmax * 8));
    LR_CHECK(keep(&hs2, (size_t)(lr::sp_sort_tiles(tmax) + 1) * 256 * 4));
    LR_CHECK(keep(&ca, (size_t)nchs * 2 * PC * 8));
    LR_CHECK(keep(&fl, (size_t)nchs * 4));
    sp_sb = lr::SpSortBufs{(uint32_t*)ki, (uint32_t*)ko, (int32_t*)pi, (int32_t*)po, (double*)xv,
                           (int32_t*)hs2, (double*)ca, (int32_t*)fl, tmax};
    sp_maxnnz = (int)maxnnz;
    sp_sorted = true;
  }
  return LR_OK;
}

namespace lr {

lr_status plan_check(const lr_matrix* Xm, int k, int p, double eps, const lr_options* opt) {
  if (!Xm || !Xm->values) return fail(LR_EINVAL, "null matrix");
  if (Xm->layout != LR_DENSE_COLMAJOR && Xm->layout != LR_CSC)
    return fail(LR_EINVAL, "unknown layout");
  if (Xm->dtype < LR_F64 || Xm->dtype > LR_BF16) return fail(LR_EINVAL, "bad dtype");
  const int64_t d = Xm->d, n = Xm->n;
  if (Xm->layout == LR_CSC) {
    if (!Xm->col_ptr || !Xm->row_idx) return fail(LR_EINVAL, "null CSC index array");
    if (d < 2 || n < 1 || Xm->nnz < 0 || Xm->nnz > 0x7fffffff)
      return fail(LR_EINVAL, "bad sizes");
  } else if (d < 2 || n < 1 || Xm->ld < d) {
    return fail(LR_EINVAL, "bad sizes");
  }
  if (!(1 <= k && k < p && p < d) || p > n || p > LR_MAX_P)
    return fail(LR_EINVAL, "need 1 <= k < p < d, p <= n, p <= 64");
  if (d > 0x7fffffff || n > 0x7fffffff) return fail(LR_EINVAL, "d and n must fit in int32");
  if (!(eps > 0)) return fail(LR_EINVAL, "eps must be positive");
  if (opt) {
    if (opt->batch < 0 || opt->batch > 8192) return fail(LR_EINVAL, "batch must be in [0, 8192]");
    if (opt->precision < LR_PREC_F64 || opt->precision > LR_PREC_MC)
      return fail(LR_EINVAL, "unknown precision");
    if ((opt->precision == LR_PREC_MC_PASS || opt->precision == LR_PREC_MC) &&
        (Xm->layout != LR_DENSE_COLMAJOR || Xm->dtype == LR_F64 || Xm->ld % 8 ||
         (uintptr_t)Xm->values % 16))
      return fail(LR_EINVAL, "matrix-core passes need dense FP32 or BF16 X with ld a multiple "
                  "of 8 and a 16-byte aligned base");
    if (opt->precision == LR_PREC_BF16_STEPS &&
        (Xm->layout != LR_DENSE_COLMAJOR || Xm->dtype != LR_BF16))
      return fail(LR_EINVAL, "BF16 matrix-core steps need dense BF16 X");
    if (opt->precision == LR_PREC_F32_STEPS &&
        (Xm->layout != LR_DENSE_COLMAJOR || Xm->dtype == LR_F64))
      return fail(LR_EINVAL, "FP32 matrix-core steps need dense FP32 or BF16 X");
    if (opt->adaptive < 0 || opt->adaptive > 1) return fail(LR_EINVAL, "adaptive must be 0 or 1");
    if (opt->norm < 0 || opt->norm > 1) return fail(LR_EINVAL, "norm must be 0 or 1");
    if (opt->accel < 0 || opt->accel > 1) return fail(LR_EINVAL, "accel must be 0 or 1");
    if (opt->fill_workspace < 0 || opt->fill_workspace > 1)
      return fail(LR_EINVAL, "fill_workspace must be 0 or 1");
    if (!(opt->shift_start >= 0) || !std::isfinite(opt->shift_start))
      return fail(LR_EINVAL, "shift_start must be a finite value >= 0");
    if (opt->accel && opt->replay)
      return fail(LR_EINVAL, "a replay schedule drives the plain inner solver only");
    if (opt->adaptive &&
        (Xm->layout != LR_DENSE_COLMAJOR || opt->precision != LR_PREC_F64 || opt->replay))
      return fail(LR_EINVAL, "adaptive partitioning needs dense X, FP64 precision, no replay");
    if (opt->replay) {
      const lr_schedule* r = opt->replay;
      if (r->outer < 0 || (r->outer > 0 && !r->epochs) || r->b < 1 || r->b > n || r->b > 8192 ||
          r->m < 1 || !(r->lambda > 0) || !(r->eta > 0))
        return fail(LR_EINVAL, "bad replay schedule");
    }
  }
  return LR_OK;
}

namespace {
// Fill the size fields of a plan for X, k, p (no allocation).
void plan_shape(lr_plan_s* pl, const lr_matrix* Xm, int k, int p, const lr_options* opt) {
  pl->sparse = Xm->layout == LR_CSC;
  pl->X = lr::XView{Xm->values, Xm->d, Xm->n, pl->sparse ? Xm->d : Xm->ld, Xm->dtype};
  pl->Xs = lr::CscView{Xm->values, Xm->col_ptr, Xm->row_idx, Xm->d, Xm->n, Xm->nnz, Xm->dtype};
  pl->k = k;
  pl->p = p;
  pl->d = Xm->d;
  pl->n = Xm->n;
  pl->bmax = std::min<int64_t>(Xm->n, 8192);
  pl->PC = lr::pad16(p);
  pl->pb.nsplit = pl->sparse ? 0 : lr::pass_nsplit(Xm->d, Xm->n);
  const int prec = opt ? opt->precision : LR_PREC_F64;
  pl->mc_pass = prec == LR_PREC_MC_PASS || prec == LR_PREC_MC;
  pl->bf16_steps = prec == LR_PREC_BF16_STEPS || (prec == LR_PREC_MC && Xm->dtype == LR_BF16);
  pl->f32_steps = prec == LR_PREC_F32_STEPS || (prec == LR_PREC_MC && Xm->dtype == LR_F32);
  pl->adaptive = opt && opt->adaptive == 1;
  pl->accel = opt && opt->accel == 1;
  pl->ldD = lr::pad_to(Xm->d, 32);
  pl->ldC = lr::pad_to(pl->bmax, 32);
}

// Device bytes the compressed-column path keeps besides the carved block: the
// row-ordered copy (column ids and values), chunk tables, head-row map, the
// chunk partial sums (at most d + nnz / SP_CHUNK chunks) and, bounded from
// above with the largest column taken as min(d, nnz) entries, the buffers of
// the sorted inner-step scatter.
size_t sparse_extra_bytes(const lr_plan_s* pl) {
  if (!pl->sparse) return 0;
  const int64_t nnz = pl->Xs.nnz, d = pl->d;
  const size_t elt = pl->Xs.dt == LR_F64 ? 8 : pl->Xs.dt == LR_F32 ? 4 : 2;
  const int64_t nch = d + nnz / lr::SP_CHUNK + 1;
  const int64_t tmax = std::min<int64_t>(pl->bmax * std::max<int64_t>(1, std::min(d, nnz)),
                                         lr::SP_SORT_CAP);
  return (size_t)nnz * (4 + elt) + (size_t)(d + 1 + nch + 1 + d + 1024) * 4 +
         (size_t)nch * pl->PC * 8 + lr::sp_sort_bytes(tmax, pl->PC);
}
}  // namespace

lr_status plan_bytes(const lr_matrix* Xm, int k, int p, const lr_options* opt, size_t* bytes) {
  LR_CHECK(plan_check(Xm, k, p, 1.0, opt));
  lr_plan_s tmp;
  tmp.owns_ws = false;
  tmp.owns_host = false;
  plan_shape(&tmp, Xm, k, p, opt);
  *bytes = tmp.carve(nullptr) + sparse_extra_bytes(&tmp);
  return LR_OK;
}

namespace {
// Fill a default-constructed plan in place: shape, replay copy, workspace
// (allocated, or carved from ws), host resources (created, or borrowed), and
// for compressed-column X the row-ordered copy.  On failure the caller
// destroys the plan.
lr_status plan_init(lr_plan_s* pl, const lr_matrix* Xm, int k, int p, double eps,
                    const lr_options* opt, hipStream_t st, void* ws, size_t ws_bytes,
                    const HostRes* host) {
  pl->st = st;
  pl->eps = eps;
  if (opt)
    pl->opt = *opt;
  else
    lowrank_options_default(&pl->opt);
  plan_shape(pl, Xm, k, p, &pl->opt);
  if (pl->opt.replay) {
    const lr_schedule* r = pl->opt.replay;
    pl->replay = true;
    pl->rsched = *r;
    pl->repochs.assign(r->epochs, r->epochs + r->outer);
    pl->rsched.epochs = nullptr;
    pl->opt.replay = nullptr;
  }
  const size_t need = pl->carve(nullptr);
  if (ws) {
    pl->owns_ws = false;
    if (ws_bytes < need) return fail(LR_EINVAL, "workspace smaller than the plan needs");
    pl->ws = ws;
  } else if (hipMalloc(&pl->ws, need) != hipSuccess) {
    (void)hipGetLastError();
    pl->ws = nullptr;
    return fail(LR_ENOMEM, "device allocation failed");
  }
  pl->carve((char*)pl->ws);
  if (pl->opt.fill_workspace && lr::fill_bytes(pl->ws, need, 0xFF, st) != hipSuccess)
    return fail(LR_EDEVICE, "workspace fill failed");
  if (host) {
    pl->owns_host = false;
    pl->hpin = host->hpin;
    for (int i = 0; i < 8; ++i) pl->ev[i] = host->ev[i];
  } else {
    LR_CHECK(host_res_create(&pl->hpin, pl->ev));
  }
  if (pl->sparse) LR_CHECK(pl->sparse_setup());
  return LR_OK;
}
}  // namespace

lr_status plan_make(lr_plan_s** out, const lr_matrix* Xm, int k, int p, double eps,
                    const lr_options* opt, hipStream_t st, void* ws, size_t ws_bytes,
                    const HostRes* host) {
  *out = nullptr;
  LR_CHECK(plan_check(Xm, k, p, eps, opt));
  lr_plan_s* pl = nullptr;
  try {
    pl = new lr_plan_s();
  } catch (...) {
    return fail(LR_ENOMEM, "host allocation failed");
  }
  const lr_status s = plan_init(pl, Xm, k, p, eps, opt, st, ws, ws_bytes, host);
  if (s != LR_OK) {
    delete pl;
    return s;
  }
  *out = pl;
  return LR_OK;
}

lr_status solve_borrowed(const lr_matrix* Xm, int k, int p, double eps, const lr_options* opt,
                         hipStream_t st, void* ws, size_t ws_bytes, const HostRes* host,
                         double* U_out, double* theta_out, lr_report* rep) {
  LR_CHECK(plan_check(Xm, k, p, eps, opt));
  if (Xm->layout != LR_DENSE_COLMAJOR)
    return fail(LR_EINVAL, "a borrowed workspace needs dense X (compressed-column plans "
                "build a row-ordered copy of X at plan time)");
  if (opt && opt->timing)
    return fail(LR_EINVAL, "timing needs the plan's own events");
  lr_plan_s pl;   // on the stack: owns neither the workspace nor the host resources
  LR_CHECK(plan_init(&pl, Xm, k, p, eps, opt, st, ws, ws_bytes, host));
  return lowrank_solve(&pl, U_out, theta_out, rep);
}

lr_status host_res_create(double** hpin, hipEvent_t* ev) {
  if (hipHostMalloc((void**)hpin, HOST_PIN_BYTES) != hipSuccess) {
    (void)hipGetLastError();
    *hpin = nullptr;
    return fail(LR_ENOMEM, "pinned host allocation failed");
  }
  for (int i = 0; i < 8; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) return fail(LR_EDEVICE, "hipEventCreate failed");
  return LR_OK;
}

void host_res_destroy(double* hpin, hipEvent_t* ev) {
  if (hpin) (void)hipHostFree(hpin);
  for (int i = 0; i < 8; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
}

}  // namespace lr

extern "C" {

const char* lowrank_status_string(lr_status s) {
  switch (s) {
    case LR_OK: return "ok";
    case LR_EINVAL: return "invalid argument";
    case LR_ENOMEM: return "out of device memory";
    case LR_ENOGAP: return "no gap between theta_k and theta_p";
    case LR_ENOCONV: return "did not converge";
    case LR_ESHIFT: return "shift not above lambda_1";
    case LR_ENOTSPD: return "Gram matrix not positive definite";
    case LR_EDEVICE: return "device error";
    case LR_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* lowrank_last_error(void) { return g_err.c_str(); }

void lowrank_options_default(lr_options* o) {
  if (!o) return;
  *o = lr_options{};
  o->seed = 0;
  o->shift_mode = 0;
  o->est_iters = 4;
  o->max_outer = 2000;
  o->max_epochs = 60;
  o->max_shift_rounds = 30;
  o->polish = 0;
  o->batch = 0;
  o->eta_scale = 1.0;
  o->tau_shift = 1e-2;
  o->replay = nullptr;
  o->timing = 0;
  o->precision = LR_PREC_F64;
  o->adaptive = 0;
  o->norm = 0;
  o->accel = 0;
  o->fill_workspace = 0;
  o->shift_start = 0.0;
}

lr_status lowrank_plan(lr_plan* out, const lr_matrix* Xm, int k, int p, double eps,
                       const lr_options* opt, void* hip_stream) {
  if (!out) return fail(LR_EINVAL, "null plan pointer");
  *out = nullptr;
  return lr::plan_make(out, Xm, k, p, eps, opt, (hipStream_t)hip_stream, nullptr, 0, nullptr);
}

lr_status lowrank_plan_bytes(const lr_matrix* X, int k, int p, const lr_options* opt,
                             size_t* bytes) {
  if (!bytes) return fail(LR_EINVAL, "null output");
  *bytes = 0;
  return lr::plan_bytes(X, k, p, opt, bytes);
}

lr_status lowrank_solve(lr_plan plan, double* U_out, double* theta_out, lr_report* rep) {
  if (!plan) return fail(LR_EINVAL, "null plan");
  try {
    return plan->adaptive ? plan->solve_adaptive(U_out, theta_out, rep)
                          : plan->solve(U_out, theta_out, rep);
  } catch (...) {
    return fail(LR_EDEVICE, "unexpected exception");
  }
}

lr_status lowrank_get_schedule(lr_plan plan, lr_schedule* out) {
  if (!plan || !out) return fail(LR_EINVAL, "null argument");
  int32_t* buf = out->epochs;
  const int32_t cap = out->n_epochs;
  *out = plan->sched;
  out->outer = (int32_t)plan->epochs.size();
  out->epochs = buf;
  out->n_epochs = cap;
  if (buf && cap > 0) {
    const int32_t c = std::min<int32_t>(cap, out->outer);
    std::memcpy(buf, plan->epochs.data(), c * sizeof(int32_t));
  }
  return LR_OK;
}

void lowrank_destroy(lr_plan plan) { delete plan; }

lr_status lowrank_op_apply_A(lr_plan plan, const double* W, double* Y, int ncols) {
  if (!plan || !W || !Y || ncols < 1 || ncols > plan->p) return fail(LR_EINVAL, "bad argument");
  plan->mc_active = plan->mc_pass;
  const lr_status s = plan->applyA(W, Y, ncols);
  plan->mc_active = false;
  LR_CHECK(s);
  LR_HIP(hipStreamSynchronize(plan->st));
  return LR_OK;
}

lr_status lowrank_op_prepare(lr_plan plan, double* w_out, uint64_t* cdf_out, double* fro2_out) {
  if (!plan) return fail(LR_EINVAL, "null plan");
  LR_CHECK(plan->prepare());
  if (w_out)
    LR_HIP(hipMemcpyAsync(w_out, plan->w, plan->n * sizeof(double), hipMemcpyDeviceToDevice,
                          plan->st));
  if (cdf_out)
    LR_HIP(hipMemcpyAsync(cdf_out, plan->cdf, (plan->n + 1) * sizeof(uint64_t),
                          hipMemcpyDeviceToDevice, plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  if (fro2_out) *fro2_out = plan->fro2;
  return LR_OK;
}

lr_status lowrank_op_sample(lr_plan plan, int32_t solve, int32_t epoch, int32_t step, int64_t b,
                            int32_t* idx_out, double* scale_out) {
  if (!plan || !idx_out || !scale_out || b < 1 || solve < 0 || epoch < 0 || step < 0 ||
      solve >= (1 << 28))
    return fail(LR_EINVAL, "bad argument");
  if (!plan->prepared) return fail(LR_EINVAL, "call lowrank_op_prepare first");
  LR_HIP(lr::sample_only(plan->n, plan->cdf, plan->opt.seed, (uint32_t)step, (uint32_t)epoch,
                         stream_word(TAG_SAMPLES, (uint32_t)solve), b, idx_out, scale_out,
                         plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  return LR_OK;
}

lr_status lowrank_op_gaussian(lr_plan plan, int32_t tag, int32_t solve, int ncols, double* S_out) {
  if (!plan || !S_out || ncols < 1 || tag < 0 || tag > 15 || solve < 0 || solve >= (1 << 28))
    return fail(LR_EINVAL, "bad argument");
  LR_HIP(lr::gaussian(S_out, plan->d, ncols, plan->opt.seed,
                      stream_word((uint32_t)tag, (uint32_t)solve), plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  return LR_OK;
}

lr_status lowrank_op_cholqr2(lr_plan plan, const double* W, double* S_out, int ncols) {
  if (!plan || !W || !S_out || ncols < 1 || ncols > plan->p) return fail(LR_EINVAL, "bad argument");
  LR_HIP(hipMemsetAsync(plan->dinfo, 0, sizeof(int), plan->st));
  LR_CHECK(plan->cholqr2(W, S_out, ncols));
  LR_CHECK(plan->check_spd());
  return LR_OK;
}

lr_status lowrank_op_eigh(lr_plan plan, const double* H, int m, double* vals_out,
                          double* vecs_out) {
  if (!plan || !H || !vals_out || !vecs_out || m < 1 || m > LR_MAX_P)
    return fail(LR_EINVAL, "bad argument");
  LR_HIP(lr::eigh(H, m, vals_out, vecs_out, plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  return LR_OK;
}

lr_status lowrank_op_estimate(lr_plan plan, int ncols, int iters, int32_t stream_index,
                              double* theta_out, double* res_out, double* V_out) {
  if (!plan || !theta_out || ncols < 2 || ncols > plan->p || iters < 0 || stream_index < 0 ||
      stream_index >= (1 << 28))
    return fail(LR_EINVAL, "bad argument");
  const int32_t saved = plan->opt.est_iters;
  plan->opt.est_iters = iters;
  double res[LR_MAX_P];
  LR_HIP(hipMemsetAsync(plan->dinfo, 0, sizeof(int), plan->st));
  const lr_status s = plan->estimate(ncols, stream_index, theta_out, res);
  plan->opt.est_iters = saved;
  LR_CHECK(s);
  if (res_out) std::memcpy(res_out, res, ncols * sizeof(double));
  if (V_out)   // estimate() leaves the Ritz vectors Sest Q in Tm2
    LR_HIP(hipMemcpyAsync(V_out, plan->Tm2, plan->d * ncols * sizeof(double),
                          hipMemcpyDeviceToDevice, plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  return LR_OK;
}

lr_status lowrank_op_power(lr_plan plan, const double* S_in, int ncols, int max_iters,
                           double tol, double* S_out, int32_t* iters_out, double* change_out) {
  if (!plan || !S_in || !S_out || ncols < 1 || ncols > plan->p || max_iters < 0 || !(tol >= 0))
    return fail(LR_EINVAL, "bad argument");
  lr_plan_s* pl = plan;
  LR_HIP(hipMemsetAsync(pl->dinfo, 0, sizeof(int), pl->st));
  LR_CHECK(pl->cholqr2(S_in, pl->S, ncols));
  int it = 0;
  double ch = -1.0;
  while (it < max_iters) {
    LR_CHECK(pl->applyA(pl->S, pl->Y, ncols));
    LR_CHECK(pl->cholqr2(pl->Y, pl->W, ncols));
    LR_CHECK(pl->subspace_change(pl->S, pl->W, ncols, &ch));
    std::swap(pl->S, pl->W);
    ++it;
    if (tol > 0 && ch <= tol) break;
  }
  LR_CHECK(pl->check_spd());
  LR_HIP(hipMemcpyAsync(S_out, pl->S, pl->d * ncols * sizeof(double), hipMemcpyDeviceToDevice,
                        pl->st));
  LR_HIP(hipStreamSynchronize(pl->st));
  if (iters_out) *iters_out = it;
  if (change_out) *change_out = ch;
  return LR_OK;
}

lr_status lowrank_op_svrg_solve(lr_plan plan, const double* S, double lambda, double eta,
                                int64_t m, int64_t b, int32_t solve, int32_t epochs,
                                double* W_out, double* res_out) {
  if (!plan || !S || !W_out || m < 1 || b < 1 || b > plan->n || epochs < 0 || solve < 0 ||
      !(lambda > 0) || !(eta > 0))
    return fail(LR_EINVAL, "bad argument");
  if (b > plan->bmax) return fail(LR_EINVAL, "minibatch larger than the plan's workspace");
  if (!plan->prepared) return fail(LR_EINVAL, "call lowrank_op_prepare first");
  std::vector<double> hist;
  int32_t e = 0;
  plan->mc_active = plan->mc_pass;
  const lr_status s = plan->svrg_solve(S, lambda, eta, m, b, solve, 0.0, epochs, &e, &hist);
  plan->mc_active = false;
  LR_CHECK(s);
  LR_HIP(hipMemcpyAsync(W_out, plan->Wt, plan->d * plan->p * sizeof(double),
                        hipMemcpyDeviceToDevice, plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  if (res_out) std::memcpy(res_out, hist.data(), hist.size() * sizeof(double));
  return LR_OK;
}

lr_status lowrank_op_acc_svrg_solve(lr_plan plan, const double* S, double lambda, double kappa,
                                    double beta, double eta, int64_t m, int64_t b, int32_t solve,
                                    int32_t epochs, double* W_out, double* res_out) {
  if (!plan || !S || !W_out || m < 1 || b < 1 || b > plan->n || epochs < 0 || solve < 0 ||
      !(lambda > 0) || !(eta > 0) || !(kappa >= 0) || !(beta >= 0 && beta < 1))
    return fail(LR_EINVAL, "bad argument");
  if (!plan->accel) return fail(LR_EINVAL, "plan made without accel = 1");
  if (b > plan->bmax) return fail(LR_EINVAL, "minibatch larger than the plan's workspace");
  if (!plan->prepared) return fail(LR_EINVAL, "call lowrank_op_prepare first");
  std::vector<double> hist;
  int32_t e = 0;
  plan->mc_active = plan->mc_pass;
  const lr_status s =
      plan->svrg_solve(S, lambda, eta, m, b, solve, 0.0, epochs, &e, &hist, -1, kappa, beta);
  plan->mc_active = false;
  LR_CHECK(s);
  LR_HIP(hipMemcpyAsync(W_out, plan->Wt, plan->d * plan->p * sizeof(double),
                        hipMemcpyDeviceToDevice, plan->st));
  LR_HIP(hipStreamSynchronize(plan->st));
  if (res_out) std::memcpy(res_out, hist.data(), hist.size() * sizeof(double));
  return LR_OK;
}

}  // extern "C"
