// Internal declarations of the NN library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/nn.h"

namespace nn {

// Number of XCDs of an MI355X; workgroups are dealt round-robin to them.
constexpr int kNumXcd = 8;

// Epilogue of a GEMM C = alpha * (A B) + E + diag * I (E optional), with an
// optional per-tile sum of |C_ij|^2 written to partials[tile] (FP64).
struct GemmArgs {
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  const void* E;  // may be null
  int64_t lde;
  int64_t M, N, K;  // real (not complex) extents of the product
  double alpha;
  double diag;
  double* partials;  // may be null
  // Split-K (only for plans with split > 1): a caller-provided buffer of
  // gemm_work_bytes() for the split partial products; null runs unsplit.
  void* work = nullptr;
  int64_t kchunk = 0;  // set by launch_gemm: k extent of one split (0: all of K)
  // Device flag (may be null): when *skip is nonzero at launch the kernel
  // returns at once without touching C or the partials (a loop whose stopping
  // rules run on the device enqueues nests past its stop as no-ops).
  const int32_t* skip = nullptr;
};

enum class Elem { F64, F32, BF16IN_F32OUT };

// Tile configurations selectable by the host (macro tile, waves, k-slab):
//   T128   128x128, 4 waves of 64x64, BK 16
//   T128W8 128x128, 8 waves of 64x32, BK 16 (two waves per SIMD)
//   T128K8 128x128, 4 waves of 64x64, BK 8, register budget for two waves/SIMD
//   T128W8K8 128x128, 8 waves of 64x32, BK 8
//   T256K8 256x128, 8 waves of 64x64, BK 8
//   T256   256x128, 8 waves of 64x64, BK 16
//   T64     64x64,  4 waves of 32x32, BK 16
//   T32     32x32,  1 wave  of 32x32, BK 16
//   T16     16x16,  4 waves each taking every fourth 64-deep k chunk, summed
//           in LDS (small products; never split)
// The environment variable NN_GEMM_TILE (one of the names above) forces one
// configuration for every GEMM, for tuning and for tests.
enum class Tile { T128, T128W8, T128K8, T128W8K8, T256K8, T256, T64, T32, T16, kCount };

struct GemmPlan {
  Tile tile;
  int tiles_m, tiles_n;
  int split = 1;  // k splits (plan_gemm_k only)
  int num_tiles() const { return tiles_m * tiles_n; }
};

// Plan (tile choice, grid) for a real M x N product.
GemmPlan plan_gemm(Elem e, int64_t M, int64_t N);
// The same plus a k split for products whose tiles cannot fill the chip
// (thin outputs, long K): each split multiplies a K/split slab range into a
// partial buffer, and a second kernel sums the partials in split order and
// applies the epilogue.  NN_GEMM_SPLIT (a power of two) forces the split.
GemmPlan plan_gemm_k(Elem e, int64_t M, int64_t N, int64_t K);
// Bytes of the partial buffer a plan_gemm_k plan needs (0 if unsplit).
size_t gemm_work_bytes(const GemmPlan& plan, Elem e, int64_t M, int64_t N);

// Enqueue C = alpha A B + E + diag I on `stream`.  `complex_b` expands B on
// the fly into the real 2K x 2N form of a complex matrix (A, C, E are then
// the interleaved real views of complex matrices, K and N real extents).
hipError_t launch_gemm(Elem e, bool complex_b, const GemmPlan& plan, const GemmArgs& a,
                       hipStream_t stream);

// BF16-input GEMM: C = alpha * A Bt^T + E + diag * I (A: M x K, Bt: N x K, BF16
// row-major; E, C FP32).  Optional outputs: C (FP32), Cbf (BF16 row-major),
// CbfT (BF16 transposed), per-tile FP64 sums of squares.
struct Bf16GemmArgs {
  const uint16_t* A;
  int64_t lda;
  const uint16_t* Bt;
  int64_t ldb;
  int64_t M, N, K;
  double alpha, diag;
  const float* E;
  int64_t lde;
  float* C;
  int64_t ldc;
  uint16_t* Cbf;
  int64_t ldcb;
  uint16_t* CbfT;
  int64_t ldct;
  double* partials;
};
GemmPlan plan_gemm_bf16(int64_t M, int64_t N);
hipError_t launch_gemm_bf16(const GemmPlan& plan, const Bf16GemmArgs& a, hipStream_t s);
// FP32/FP64 -> BF16, optionally also the transposed copy (dst or dstT may be null).
hipError_t launch_cast_bf16(bool f64, const void* src, int64_t lds, uint16_t* dst, int64_t ldd,
                            uint16_t* dstT, int64_t ldt, int64_t rows, int64_t cols,
                            hipStream_t s);

// X_0 prologue.  scal[0] <- den (||A||_1 ||A||_inf or Re Tr A).
hipError_t launch_den_transpose(nn_dtype dt, const void* A, int64_t lda, int64_t n, double* part,
                                double* scal, hipStream_t s);
hipError_t launch_den_trace(nn_dtype dt, const void* A, int64_t lda, int64_t n, double* scal,
                            hipStream_t s);
size_t den_partials_elems(int64_t n);
// X = A^H / den  or  X = I / den, den read from scal[0] on the device.
hipError_t launch_x0_transpose(nn_dtype dt, const void* A, int64_t lda, void* X, int64_t ldx,
                               int64_t n, const double* scal, hipStream_t s);
hipError_t launch_x0_identity(nn_dtype dt, void* X, int64_t ldx, int64_t n, const double* scal,
                              hipStream_t s);

// Start iterate X_0 for every x0 choice except NN_X0_GIVEN (nn_start.hip):
// the scale den lands in scal[0] (not finite: NONFINITE; <= 0: DIVERGED).
// denpart: den_partials_elems(n) doubles; pw: start_scratch_doubles(n).
constexpr int kPowerMaxK = 64;
size_t start_scratch_doubles(int64_t n);
hipError_t launch_start(nn_dtype dt, int x0, int power_k, const void* A, int64_t lda, void* X,
                        int64_t ldx, int64_t n, double* denpart, double* pw, double* scal,
                        hipStream_t s);

// The SplitMix64 power-iteration vector (real values; zero imaginary parts
// when cplx) and its squared entries; out[0] = mult * sqrt(sum part[0..count)).
hipError_t launch_power_vector(bool cplx, double* x, double* rowsq, int64_t n, hipStream_t s);
hipError_t launch_norm_reduce(const double* part, int64_t count, double mult, double* out,
                              hipStream_t s);

// Sum `count` FP64 partials in a fixed order; out[0] <- sqrt(sum / n_rows).
hipError_t launch_rms_reduce(const double* partials, int count, int64_t n_rows, double* out,
                             hipStream_t s);

// Control block of a tolerance-mode loop whose stopping rules run on the
// device.  `done` is the skip flag of the loop's GEMMs; when it is set,
// status/iters/rms_ret hold the outcome, with the meanings of the host loop.
struct DevCtl {
  int32_t done;
  int32_t status;
  int32_t iters;
  int32_t last_k;   // index of the last residual the rules were applied to
  double rms_prev;  // rms of the previous residual that passed every rule
  double rms_ret;   // rms of the returned iterate
};
// ctl <- {done 0, status OK, iters 0, last_k -1, NaN, NaN} (a kernel, not a
// memset, so the loop can be captured).  With den non-null, the start scale
// den[0] is tested first: not finite -> done with NONFINITE, <= 0 -> done
// with DIVERGED.
hipError_t launch_ctl_init(DevCtl* ctl, const double* den, hipStream_t s);
// Unless ctl->done: out[0] <- rms of nest k's residual (the same fixed-order
// sum as launch_rms_reduce, so the same bits), then the rules of the host
// loop for index k with tol and max_iter (stagnation test with sqrt(n_rows)).
hipError_t launch_rms_control(const double* partials, int count, int64_t n_rows, double* out,
                              DevCtl* ctl, int k, double tol, int max_iter, hipStream_t s);

// Element-wise copies/casts of an n x n (real extents rows x cols) matrix.
hipError_t launch_copy(size_t elem_bytes, const void* src, int64_t lds, void* dst, int64_t ldd,
                       int64_t rows, int64_t cols_bytes, hipStream_t s);
hipError_t launch_cast_f64_f32(const double* src, int64_t lds, float* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_cast_f32_f64(const float* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_cast_f64_bf16(const double* src, int64_t lds, uint16_t* dst, int64_t ldd,
                                int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_cast_f32_bf16(const float* src, int64_t lds, uint16_t* dst, int64_t ldd,
                                int64_t rows, int64_t cols, hipStream_t s);

// Sum of squares of an rows x cols real matrix into out[0] (fixed order).
hipError_t launch_sumsq(const void* src, bool f64, int64_t ld, int64_t rows, int64_t cols,
                        double* part, double* out, hipStream_t s);

// Batched persistent path: plan kernel + persistent kernel on stream s.
// Matrices of size <= wave_max_k (<= 32) get one wave each; grid workgroups.
size_t batched_ws_bytes(int32_t batch);
size_t batched_lds_bytes(nn_dtype dt, int max_n, int wave_max_k, int depth);
hipError_t batched_allow_lds();  // raise the dynamic LDS limit (call outside capture)
// LDS of one CU, and the dynamic LDS limit the batched kernels are given.
constexpr size_t kBatchedLdsCu = 160 * 1024;
constexpr size_t kBatchedDynLds = 150 * 1024;
// Static LDS of the persistent kernel (from the compiled kernel's attributes).
size_t batched_static_lds();
// The largest one-wave size limit <= wave_max_k (stepping 32 -> 16 -> 8 -> 0)
// whose LDS fits one workgroup: dynamic part <= kBatchedDynLds and dynamic +
// static <= kBatchedLdsCu.  (Complex matrices at depth >= 3 with one-wave
// matrices up to 32 would need 204 KB.)
int batched_fit_wave_max_k(nn_dtype dt, int max_n, int wave_max_k, int depth);
// Arguments of one batched launch.  Matrix b: A at element offset offsets[b],
// X at xoffsets[b] (offsets if null), size sizes[b].  iters > 0: exactly that
// many nests; iters == 0: tolerance mode with tols[b] (tol if null) and
// maxits[b] (max_iter if null).  x0: TRANSPOSE, SCALED_IDENTITY or GIVEN (X
// holds X_0 on entry).
struct BatchedArgs {
  nn_dtype dt = NN_C64;
  const void* A = nullptr;
  void* X = nullptr;
  const int64_t* offsets = nullptr;
  const int64_t* xoffsets = nullptr;
  const int32_t* sizes = nullptr;
  const double* tols = nullptr;
  const int32_t* maxits = nullptr;
  int32_t batch = 0, max_n = 0;
  int depth = 2, x0 = 0, iters = 0;
  double tol = 0.0;
  int max_iter = 0;
  int wave_max_k = 16;
  int quad_max_k = 0;  // set by launch_batched
  void* ws = nullptr;
  nn_info_dev* info = nullptr;
  int grid = 1;
};
hipError_t launch_batched(const BatchedArgs& a, hipStream_t s);
// The largest blocks-per-wave count any matrix of size <= max_n takes (one
// wave up to wave_max_k, a whole workgroup above): 1, 2, 4 or 8.
int batched_max_nb(bool cplx, int max_n, int wave_max_k);

// Upper bound of max_iter for the batched tolerance mode (bounds the
// persistent kernel's run time).
constexpr int kBatchedMaxIter = 4096;

inline size_t elem_size(nn_dtype d) {
  switch (d) {
    case NN_F64: return 8;
    case NN_F32: return 4;
    case NN_C64: return 8;
    case NN_C128: return 16;
  }
  return 0;
}
inline bool is_complex(nn_dtype d) { return d == NN_C64 || d == NN_C128; }
inline bool is_double(nn_dtype d) { return d == NN_F64 || d == NN_C128; }

// Tuned configuration of the batched kernel for one (dtype, max_n).
struct BatchedTune {
  int dtype = -1, max_n = 0;
  int wave_max_k = 16;
  int wg_per_cu = 1;
};

// The instantiated graph of the last batched call and its arguments.
struct BatchedGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* A = nullptr;
  void* X = nullptr;
  const int64_t* offsets = nullptr;
  const int32_t* sizes = nullptr;
  void* ws = nullptr;
  nn_info_dev* info = nullptr;
  int32_t batch = 0, max_n = 0;
  int dtype = -1, depth = 0, x0 = 0, iters = 0, wave_max_k = 0, grid = 0;
  double tol = 0.0;
  int max_iter = 0;
};

// Uncaptured batched launch with the configuration of ctx's table for
// (a.dt, 64); fills a.wave_max_k and a.grid (nn_batched_api.cpp).
hipError_t launch_batched_direct(nn_ctx* ctx, BatchedArgs a, hipStream_t s);

}  // namespace nn

constexpr int kTimedGemms = 1024;
constexpr int kTuneSlots = 8;

struct nn_ctx {
  int device = 0;
  int num_cus = 256;
  char arch[64] = {0};  // gcnArchName of the device (autotune cache key)
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  double* host = nullptr;            // pinned read-back slots
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  hipEvent_t* ev_gemm = nullptr;  // 2 * kTimedGemms events, created on first timed call
  nn::BatchedTune tune[kTuneSlots];
  nn::BatchedGraph bgraph;
  void* scratch = nullptr;  // device address of this device's static scratch array
};
