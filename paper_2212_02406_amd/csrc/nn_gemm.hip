// nn_gemm.hip — MFMA GEMM with the fused epilogues of one NN nest (gfx950).
//
// One nest of the Nested Neumann iteration (arXiv 2212.02406, Sec. II-D
// Theorem; Algorithm 1) is d + 1 dense products.  All of them are
//     C = alpha * (A B) + E + diag * I
// with (alpha, E, diag) = (-1, -, 1) for the residual R = I - A X,
// (1, R, 0) for a Horner step U' = R + R U, and (1, X, 0) for the update
// X' = X + X U.  The identity is never stored; it is added on the diagonal in
// the epilogue.  The residual launch also writes one FP64 partial sum of
// |C_ij|^2 per output tile into a fixed slot (no atomics), which a second
// kernel reduces in a fixed order, so rms is bitwise reproducible.
//
// Kernel structure (CDNA4, wave64):
//  * macro tile BM x BN per workgroup, WM x WN waves, each wave owns a
//    (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA blocks
//    (v_mfma_f64_16x16x4_f64 for FP64, v_mfma_f32_16x16x4_f32 for FP32);
//  * A and B k-slabs of depth BK are staged global -> registers -> LDS with
//    two LDS buffers, so one barrier per slab suffices and the next slab's
//    global loads are in flight while the current one feeds the MFMAs;
//  * LDS rows are padded by 16 bytes, which makes the 16-lane fragment reads
//    bank-conflict free and keeps 16-byte vector stores aligned;
//  * workgroup -> tile mapping is XCD-aware (each of the 8 XCDs gets a
//    contiguous range of tiles, so the tiles sharing A and B panels share an
//    L2) and grouped by GROUP_M tile rows inside that range.
//  * complex matrices: C = A B in complex arithmetic equals the real product
//    of the interleaved A (M x 2K) with the real 2K x 2N form of B whose row
//    2k is B's row k as stored and row 2k+1 is the same row with each pair
//    (re, im) replaced by (-im, re).  That expansion is done while staging B.
#include <stdlib.h>
#include <string.h>

#include "nn_internal.h"

namespace nn {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Both 16x16x4 MFMAs take A[m][k] from lane m + 16 k and B[k][n] from lane
// n + 16 k, and return column n = lane % 16 of D.  They differ in the rows
// a lane's four results belong to (measured on gfx950): FP32 gives rows
// 4 (lane / 16) + t, FP64 gives rows lane / 16 + 4 t, t = 0..3.
template <>
struct Mfma<double> {
  using acc_t = d4_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return lk + 4 * t; }
};
template <>
struct Mfma<float> {
  using acc_t = f4_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int t) { return 4 * lk + t; }
};

template <typename T, int V>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecOf<T, 1> {
  typedef T type;
};

template <typename T, int V>
__device__ __forceinline__ T& lane_of(typename VecOf<T, V>::type& v, int e) {
  return reinterpret_cast<T*>(&v)[e];
}

constexpr int kGroupM = 8;

// Padding (elements) of a Bs row.  The four lane groups of a B fragment read
// rows KQ apart; the row offset between consecutive groups is placed half the
// 64 banks away for 8-byte elements (a 64-lane ds_read_b64 is served 32 lanes
// at a time) and a quarter away for 4-byte elements (64 lanes at once), so the
// groups do not collide.  Rows stay 16-byte multiples for the vector stores.
constexpr int pick_padb(int bn, int kq, int esz) {
  const int words = esz / 4, target = esz == 8 ? 32 : 16, step = 16 / esz;
  for (int p = step; p < 64; p += step)
    if ((kq * (bn + p) * words) % 64 == target) return p;
  return step;
}

// Source of the zeros loaded for out-of-range elements (read only).
__device__ __attribute__((aligned(16))) const double kZero16[2] = {0.0, 0.0};

// Load from global memory through an address-space-1 pointer.  The operand
// addresses are chosen by a select between the matrix and kZero16; without
// the cast the compiler emits flat loads, which also count against the LDS
// wait counter, so every wait for the LDS fragment reads would wait for the
// global prefetch as well.
template <typename V>
__device__ __forceinline__ V load_global(uintptr_t addr) {
  return *reinterpret_cast<const __attribute__((address_space(1))) V*>(addr);
}

__device__ __forceinline__ int xcd_remap(int bid, int nwg) {
  const int q = nwg / kNumXcd, r = nwg % kNumXcd;
  const int x = bid % kNumXcd, local = bid / kNumXcd;
  return x * q + (x < r ? x : r) + local;
}

__device__ __forceinline__ void grouped_tile(int tile, int tm, int tn, int& pm, int& pn) {
  const int group = kGroupM * tn;
  const int gid = tile / group;
  const int first = gid * kGroupM;
  const int gsize = (tm - first) < kGroupM ? (tm - first) : kGroupM;
  const int in = tile - gid * group;
  pm = first + in % gsize;
  pn = in / gsize;
}

// EXACT: M, N, K are multiples of BM, BN, BK (every tile interior, no
// bounds checks anywhere).
template <typename T, int BM, int BN, int BK, int WM, int WN, int OCC, int VEC, bool CPLX,
          bool EXACT>
__global__ void __launch_bounds__(WM* WN * 64) __attribute__((amdgpu_waves_per_eu(OCC)))
    gemm_kernel(GemmArgs p, int tiles_m, int tiles_n) {
  if (p.skip && *p.skip) return;  // uniform: the whole workgroup leaves
  constexpr int NT = WM * WN * 64;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int PAD = 16 / (int)sizeof(T);
  constexpr int KQ = BK / 4;     // k values per lane and slab (see compute)
  constexpr int LAS = BK + PAD;  // As row stride ([m][k] layout), 16-byte multiple
  // Bs row stride ([k][n] layout): lane groups read rows KQ apart, padded so
  // the four groups of a fragment read land in different banks
  constexpr int LBS = BN + pick_padb(BN, KQ, (int)sizeof(T));
  constexpr int A_VPR = BK / VEC, B_VPR = BN / VEC;
  // vectors per slab, and per thread (the last round may cover only some
  // waves when a slab holds fewer vectors than the workgroup has threads)
  constexpr int A_TOT = BM * A_VPR, B_TOT = BK * B_VPR;
  constexpr int A_LOADS = (A_TOT + NT - 1) / NT, B_LOADS = (B_TOT + NT - 1) / NT;
  static_assert(A_TOT % 64 == 0 && B_TOT % 64 == 0, "whole waves per load round");
  static_assert(BK % 4 == 0 && WTM % 16 == 0 && WTN % 16 == 0, "mfma shape");
  static_assert(!CPLX || VEC % 2 == 0, "complex staging needs pairs");
  using acc_t = typename Mfma<T>::acc_t;
  using vec_t = typename VecOf<T, VEC>::type;

  __shared__ __attribute__((aligned(16))) T As[2][BM * LAS];
  __shared__ __attribute__((aligned(16))) T Bs[2][BK * LBS];
  __shared__ double red[WM * WN];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  int pm, pn;
  const int ntile = tiles_m * tiles_n;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int sidx = bid / ntile;  // k split of this workgroup (0 when unsplit)
  grouped_tile(bid - sidx * ntile, tiles_m, tiles_n, pm, pn);
  const int64_t m0 = (int64_t)pm * BM, n0 = (int64_t)pn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  // k range [kbeg, kend): a multiple of BK wide except at the end of K
  const int64_t kbeg = p.kchunk ? (int64_t)sidx * p.kchunk : 0;
  const int64_t kend = p.kchunk ? (kbeg + p.kchunk < K ? kbeg + p.kchunk : K) : K;
  const T* __restrict__ A = static_cast<const T*>(p.A);
  const T* __restrict__ B = static_cast<const T*>(p.B);

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};

  vec_t ra[A_LOADS], rb[B_LOADS];

  // Global -> register staging, branch-free: an out-of-range vector is read
  // from a 16-byte all-zero device array instead of the matrix, so nothing
  // consumes the loaded registers until they are stored to LDS after the
  // current slab's MFMAs (the loads stay in flight across the compute).  The
  // vector path is chosen by the host only when K, N and the leading
  // dimensions are multiples of VEC, so a vector is wholly in or out.
  const uintptr_t zaddr = reinterpret_cast<uintptr_t>(kZero16);
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int v = tid + i * NT;
      if (A_TOT % NT != 0 && v >= A_TOT) break;
      const int r = v / A_VPR, c = (v % A_VPR) * VEC;
      const int64_t gr = m0 + r, gc = k0 + c;
      const bool ok = gr < M && gc < K;
      const uintptr_t src = reinterpret_cast<uintptr_t>(A + gr * p.lda + gc);
      ra[i] = load_global<vec_t>(ok ? src : zaddr);
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int v = tid + i * NT;
      if (B_TOT % NT != 0 && v >= B_TOT) break;
      const int r = v / B_VPR, c = (v % B_VPR) * VEC;
      const int64_t gr = k0 + r, gc = n0 + c;
      const int64_t srow = CPLX ? (gr >> 1) : gr;
      const bool ok = gr < K && gc < N;
      const uintptr_t src = reinterpret_cast<uintptr_t>(B + srow * p.ldb + gc);
      rb[i] = load_global<vec_t>(ok ? src : zaddr);
    }
  };

  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LOADS; ++i) {
      const int v = tid + i * NT;
      if (A_TOT % NT != 0 && v >= A_TOT) break;
      const int r = v / A_VPR, c = (v % A_VPR) * VEC;
      *reinterpret_cast<vec_t*>(&As[buf][r * LAS + c]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_LOADS; ++i) {
      const int v = tid + i * NT;
      if (B_TOT % NT != 0 && v >= B_TOT) break;
      const int r = v / B_VPR, c = (v % B_VPR) * VEC;
      vec_t x = rb[i];
      if constexpr (CPLX) {
        // odd rows of the real form of a complex B: (re, im) -> (-im, re);
        // the slab origin is a multiple of BK (even), so r's parity is the row's
        if (r & 1) {
#pragma unroll
          for (int e = 0; e < VEC; e += 2) {
            const T re = lane_of<T, VEC>(x, e), im = lane_of<T, VEC>(x, e + 1);
            lane_of<T, VEC>(x, e) = -im;
            lane_of<T, VEC>(x, e + 1) = re;
          }
        }
      }
      *reinterpret_cast<vec_t*>(&Bs[buf][r * LBS + c]) = x;
    }
  };

  // k order inside a slab: at MFMA step kk, lane group lk = lane / 16
  // supplies k = lk * KQ + kk (for A and B alike, so every k of the slab is
  // summed once).  A lane's A operands of the whole slab are then KQ
  // consecutive elements of one LDS row: one wide read per fragment.
  using kvec_t = typename VecOf<T, KQ>::type;
  const int lr = lane & 15, lk = lane >> 4;
  auto compute = [&](int buf) {
    const T* as = As[buf] + (wm * WTM + lr) * LAS + lk * KQ;
    const T* bs = Bs[buf] + lk * KQ * LBS + wn * WTN + lr;
    kvec_t av[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) av[i] = *reinterpret_cast<const kvec_t*>(as + i * 16 * LAS);
#pragma unroll
    for (int kk = 0; kk < KQ; ++kk) {
      T bf[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = bs[kk * LBS + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = Mfma<T>::run(lane_of<T, KQ>(av[i], kk), bf[j], acc[i][j]);
    }
  };

  // Exact tiling needs no bounds checks: a thread's load addresses are a
  // wave-uniform slab base plus a fixed 32-bit element offset per load, so
  // the slab loop spends no vector instructions on addresses.
  uint32_t oa[A_LOADS], ob[B_LOADS];
#pragma unroll
  for (int i = 0; i < A_LOADS; ++i) {
    const int v = tid + i * NT;
    const int r = v / A_VPR, c = (v % A_VPR) * VEC;
    oa[i] = (uint32_t)(r * p.lda + c);
  }
#pragma unroll
  for (int i = 0; i < B_LOADS; ++i) {
    const int v = tid + i * NT;
    const int r = v / B_VPR, c = (v % B_VPR) * VEC;
    ob[i] = (uint32_t)((CPLX ? (r >> 1) : r) * p.ldb + c);
  }
  auto load = [&](int64_t k0) {
    if constexpr (EXACT) {
      const T* a0 = A + m0 * p.lda + k0;
      const T* b0 = B + (CPLX ? (k0 >> 1) : k0) * p.ldb + n0;
#pragma unroll
      for (int i = 0; i < A_LOADS; ++i) {
        if (A_TOT % NT != 0 && tid + i * NT >= A_TOT) break;
        ra[i] = load_global<vec_t>(reinterpret_cast<uintptr_t>(a0 + oa[i]));
      }
#pragma unroll
      for (int i = 0; i < B_LOADS; ++i) {
        if (B_TOT % NT != 0 && tid + i * NT >= B_TOT) break;
        rb[i] = load_global<vec_t>(reinterpret_cast<uintptr_t>(b0 + ob[i]));
      }
    } else {
      gload(k0);
    }
  };

  // Steady state without conditionals: prefetch slab kt+1 into registers,
  // multiply slab kt from LDS, store slab kt+1 into the other LDS buffer.
  // FP32: each slab's fragment reads and MFMAs run at raised wave priority
  // (s_setprio 1), so the two workgroups on a CU do not interleave them with
  // each other's stores (N = 8192: 7.84 -> 7.53 ms per product, the same
  // bits).  For FP64 the same change cost 13% (15.4 -> 17.4 ms): it is left
  // out there.
  constexpr bool kPrio = sizeof(T) == 4;
  const int nk = (int)((kend - kbeg + BK - 1) / BK);
  load(kbeg);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk - 1; ++kt) {
    load(kbeg + (int64_t)(kt + 1) * BK);
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
    compute(kt & 1);
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
    sstore((kt + 1) & 1);
    __syncthreads();
  }
  compute((nk - 1) & 1);

  if (p.work) {
    // split-K: the raw partial product of this k range, row-major M x N
    T* __restrict__ Wp = static_cast<T*>(p.work) + (int64_t)sidx * M * N;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int64_t c = n0 + wn * WTN + j * 16 + lr;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int64_t r = m0 + wm * WTM + i * 16 + Mfma<T>::row(lk, t);
          if (EXACT || (r < M && c < N)) Wp[r * N + c] = acc[i][j][t];
        }
      }
    }
    return;
  }

  // Epilogue: C = alpha * acc + E + diag * I, and the tile's sum of squares.
  T* __restrict__ C = static_cast<T*>(p.C);
  const T* __restrict__ E = static_cast<const T*>(p.E);
  const T alpha = (T)p.alpha, diag = (T)p.diag;
  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t c = n0 + wn * WTN + j * 16 + lr;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t r = m0 + wm * WTM + i * 16 + Mfma<T>::row(lk, t);
        if (EXACT || (r < M && c < N)) {
          T v = alpha * acc[i][j][t];
          if (E) v += E[r * p.lde + c];
          if (CPLX ? (c == 2 * r) : (c == r)) v += diag;
          C[r * p.ldc + c] = v;
          ss += (double)v * (double)v;
        }
      }
    }
  }
  if (p.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < WM * WN; ++w) t += red[w];
      p.partials[pm * tiles_n + pn] = t;
    }
  }
}

// Small products (n up to a few hundred), where 32x32 tiles leave most of the
// 256 CUs idle and a single wave per tile waits out every load: one 16x16
// output tile per workgroup, its k range dealt to four waves in chunks of 64
// (chunk c to wave c mod 4).  A chunk needs no LDS staging: at MFMA step j
// lane (r, q) = (lane % 16, lane / 16) supplies A[m0+r][k0+16q+j] and
// B[k0+16q+j][n0+r], so a lane's 16 A operands are one contiguous row run
// (vector loads) and the 16 lanes of a B load read one contiguous row run.
// The four waves' accumulators are summed through LDS in wave order by wave
// 0, which applies the epilogue and writes the tile's sum of squares.
// EXACT: M, N multiples of 16, K of 64, A rows 16-byte aligned (no checks).
constexpr int kSmallChunk = 64;

template <typename T, bool CPLX, bool EXACT>
__global__ void __launch_bounds__(256) gemm_small_kernel(GemmArgs p, int tiles_m, int tiles_n) {
  // Wave 0 loads the epilogue's E values before the operands, so that round
  // trip overlaps the operand loads instead of following the LDS sum (the
  // kernel is bound by load latency, not arithmetic).  The device-stop flag
  // is the same for every wave: each wave leaves before the workgroup barrier
  // when it is set.
  const int skipv = p.skip ? *p.skip : 0;
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte vector
  typedef T vec_t __attribute__((ext_vector_type(V)));
  __shared__ acc_t red[3][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  int pm, pn;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  grouped_tile(bid, tiles_m, tiles_n, pm, pn);
  const int64_t m0 = (int64_t)pm * 16, n0 = (int64_t)pn * 16;
  const int64_t M = p.M, N = p.N, K = p.K;
  const T* __restrict__ A = static_cast<const T*>(p.A);
  const T* __restrict__ B = static_cast<const T*>(p.B);
  const int64_t arow = m0 + lr, bcol = n0 + lr;
  const bool arow_ok = EXACT || arow < M, bcol_ok = EXACT || bcol < N;
  const T* __restrict__ E = static_cast<const T*>(p.E);
  T ev[4] = {T(0), T(0), T(0), T(0)};
  if (wave == 0 && E) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t r = m0 + Mfma<T>::row(lq, t);
      if (EXACT || (r < M && bcol < N)) ev[t] = E[r * p.lde + bcol];
    }
  }

  acc_t acc = acc_t{};
  const int64_t nchunks = (K + kSmallChunk - 1) / kSmallChunk;
  for (int64_t c = wave; c < nchunks; c += 4) {
    const int64_t kb = c * kSmallChunk + 16 * lq;  // this lane's first k
    T a[16], b[16];
    if constexpr (EXACT) {
      const vec_t* ap = reinterpret_cast<const vec_t*>(A + arow * p.lda + kb);
#pragma unroll
      for (int v = 0; v < 16 / V; ++v) {
        const vec_t x = ap[v];
#pragma unroll
        for (int e = 0; e < V; ++e) a[v * V + e] = x[e];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t k = kb + j;
        a[j] = (arow_ok && k < K) ? A[arow * p.lda + k] : T(0);
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t k = kb + j;
      if constexpr (CPLX) {
        // real form of a complex B: row 2s is row s as stored, row 2s+1 is
        // row s with (re, im) -> (-im, re)
        const T* row = B + (k >> 1) * p.ldb;
        T v = T(0);
        if (bcol_ok && (EXACT || k < K)) {
          if (!(k & 1)) v = row[bcol];
          else v = (bcol & 1) ? row[bcol - 1] : -row[bcol + 1];
        }
        b[j] = v;
      } else {
        b[j] = (bcol_ok && (EXACT || k < K)) ? B[k * p.ldb + bcol] : T(0);
      }
    }
    if (skipv) return;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc = Mfma<T>::run(a[j], b[j], acc);
  }
  if (skipv) return;  // a wave with no chunk

  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w) acc += red[w][lane];

  T* __restrict__ C = static_cast<T*>(p.C);
  const T alpha = (T)p.alpha, diag = (T)p.diag;
  double ss = 0.0;
  const int64_t c = bcol;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t r = m0 + Mfma<T>::row(lq, t);
    if (EXACT || (r < M && c < N)) {
      T v = alpha * acc[t];
      if (E) v += ev[t];
      if (CPLX ? (c == 2 * r) : (c == r)) v += diag;
      C[r * p.ldc + c] = v;
      ss += (double)v * (double)v;
    }
  }
  if (p.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) p.partials[pm * tiles_n + pn] = ss;
  }
}

template <typename T, bool CPLX>
hipError_t launch_small(const GemmPlan& plan, const GemmArgs& a, hipStream_t s) {
  const int ntile = plan.num_tiles();
  if (ntile <= 0) return hipSuccess;
  const size_t ab = reinterpret_cast<uintptr_t>(a.A);
  const bool exact = a.M % 16 == 0 && a.N % 16 == 0 && a.K % kSmallChunk == 0 && ab % 16 == 0 &&
                     (a.lda * (int64_t)sizeof(T)) % 16 == 0;
  if (exact)
    hipLaunchKernelGGL((gemm_small_kernel<T, CPLX, true>), dim3(ntile), dim3(256), 0, s, a,
                       plan.tiles_m, plan.tiles_n);
  else
    hipLaunchKernelGGL((gemm_small_kernel<T, CPLX, false>), dim3(ntile), dim3(256), 0, s, a,
                       plan.tiles_m, plan.tiles_n);
  return hipGetLastError();
}

// Split-K epilogue, kSplitChunks workgroups per output tile (each a band of
// the tile's rows): C = alpha * sum_s W_s + E + diag * I with the partials
// summed in split order; each band's sum of squares goes to ssbuf and
// splitk_tile_ss adds a tile's bands in order into partials[tile] (the
// unsplit kernel's indexing).
constexpr int kSplitChunks = 8;

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) splitk_epilogue(GemmArgs p, int split, int bm, int bn,
                                                       int tiles_n, double* ssbuf) {
  if (p.skip && *p.skip) return;
  __shared__ double red[256];
  const int tile = blockIdx.x / kSplitChunks, band = blockIdx.x % kSplitChunks;
  const int rows = bm / kSplitChunks;
  const int64_t m0 = (int64_t)(tile / tiles_n) * bm + band * rows;
  const int64_t n0 = (int64_t)(tile % tiles_n) * bn;
  const int64_t M = p.M, N = p.N;
  const T* __restrict__ Wp = static_cast<const T*>(p.work);
  T* __restrict__ C = static_cast<T*>(p.C);
  const T* __restrict__ E = static_cast<const T*>(p.E);
  const T alpha = (T)p.alpha, diag = (T)p.diag;
  double ss = 0.0;
  for (int e = threadIdx.x; e < rows * bn; e += 256) {
    const int64_t r = m0 + e / bn, c = n0 + e % bn;
    if (r < M && c < N) {
      T v = T(0);
      for (int sp = 0; sp < split; ++sp) v += Wp[((int64_t)sp * M + r) * N + c];
      v = alpha * v;
      if (E) v += E[r * p.lde + c];
      if (CPLX ? (c == 2 * r) : (c == r)) v += diag;
      C[r * p.ldc + c] = v;
      ss += (double)v * (double)v;
    }
  }
  if (p.partials) {
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) ssbuf[blockIdx.x] = red[0];
  }
}

__global__ void __launch_bounds__(256) splitk_tile_ss(const double* ssbuf, int ntile,
                                                      double* partials) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ntile) return;
  double v = 0.0;
  for (int b = 0; b < kSplitChunks; ++b) v += ssbuf[t * kSplitChunks + b];
  partials[t] = v;
}

struct TileShape {
  int bm, bn;
};
inline TileShape shape_of(Tile t) {
  switch (t) {
    case Tile::T128:
    case Tile::T128W8:
    case Tile::T128K8:
    case Tile::T128W8K8: return {128, 128};
    case Tile::T256K8:
    case Tile::T256: return {256, 128};
    case Tile::T64: return {64, 64};
    case Tile::T16: return {16, 16};
    case Tile::T32:
    case Tile::kCount: return {32, 32};
  }
  return {32, 32};
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int OCC, int VEC, bool CPLX>
hipError_t launch_one(const GemmPlan& plan, const GemmArgs& a, hipStream_t s) {
  const int ntile = plan.num_tiles();
  if (ntile <= 0) return hipSuccess;
  // k split: whole slabs per split and no empty split
  GemmArgs b = a;
  int split = 1;
  b.kchunk = 0;
  if (a.work && plan.split > 1) {
    const int64_t slabs = (a.K + BK - 1) / BK;
    const int64_t per = (slabs + plan.split - 1) / plan.split;
    split = (int)((slabs + per - 1) / per);
    if (split > 1) b.kchunk = per * BK;
  }
  if (split == 1) b.work = nullptr;
  const int grid = ntile * split;
  // every tile interior: the kernel without bounds checks
  const bool exact = a.M % BM == 0 && a.N % BN == 0 && a.K % BK == 0;
  if (exact)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, WM, WN, OCC, VEC, CPLX, true>), dim3(grid),
                       dim3(WM * WN * 64), 0, s, b, plan.tiles_m, plan.tiles_n);
  else
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, WM, WN, OCC, VEC, CPLX, false>), dim3(grid),
                       dim3(WM * WN * 64), 0, s, b, plan.tiles_m, plan.tiles_n);
  if (split > 1) {
    static_assert(BM % kSplitChunks == 0, "row bands of a tile");
    double* ssbuf = reinterpret_cast<double*>(static_cast<char*>(a.work) +
                                              (size_t)split * a.M * a.N * sizeof(T));
    hipLaunchKernelGGL((splitk_epilogue<T, CPLX>), dim3(ntile * kSplitChunks), dim3(256), 0, s, a,
                       split, BM, BN, plan.tiles_n, ssbuf);
    if (a.partials)
      hipLaunchKernelGGL(splitk_tile_ss, dim3((ntile + 255) / 256), dim3(256), 0, s, ssbuf, ntile,
                         a.partials);
  }
  return hipGetLastError();
}

template <typename T, int VEC, bool CPLX>
hipError_t launch_tile(const GemmPlan& plan, const GemmArgs& a, hipStream_t s) {
  switch (plan.tile) {
    case Tile::T16: return launch_small<T, CPLX>(plan, a, s);
    case Tile::T128: return launch_one<T, 128, 128, 16, 2, 2, 1, VEC, CPLX>(plan, a, s);
    case Tile::T128W8: return launch_one<T, 128, 128, 16, 2, 4, 2, VEC, CPLX>(plan, a, s);
    case Tile::T128K8: return launch_one<T, 128, 128, 8, 2, 2, 2, VEC, CPLX>(plan, a, s);
    case Tile::T128W8K8: return launch_one<T, 128, 128, 8, 2, 4, 2, VEC, CPLX>(plan, a, s);
    case Tile::T256K8: return launch_one<T, 256, 128, 8, 4, 2, 2, VEC, CPLX>(plan, a, s);
    case Tile::T256: return launch_one<T, 256, 128, 16, 4, 2, 2, VEC, CPLX>(plan, a, s);
    case Tile::T64: return launch_one<T, 64, 64, 16, 2, 2, 1, VEC, CPLX>(plan, a, s);
    case Tile::T32:
    case Tile::kCount: return launch_one<T, 32, 32, 16, 1, 1, 1, VEC, CPLX>(plan, a, s);
  }
  return hipErrorInvalidValue;
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }


bool tile_override(Tile* t) {
  const char* v = getenv("NN_GEMM_TILE");
  if (!v) return false;
  const char* names[] = {"T128", "T128W8", "T128K8", "T128W8K8", "T256K8", "T256", "T64", "T32",
                         "T16"};
  for (int i = 0; i < (int)Tile::kCount; ++i) {
    if (strcmp(v, names[i]) == 0) {
      *t = static_cast<Tile>(i);
      return true;
    }
  }
  return false;
}

}  // namespace

// Largest output (M x N real elements) for which the small-product kernel
// beats the 32x32 and 64x64 tiles on gfx950 (square products, ten depth-2
// nests, microseconds per GEMM): FP64 n = 256: 7.3 against 18.8 (T32);
// n = 640: 34.4 against 39.1; n = 768: 49.0 against 46.8.  FP32 n = 256: 7.7
// against 13.5; n = 768: 27.2 against 33.1; n = 1024: 54.4 against 42.4.
// Longer k extents (thin products over a large n) keep the split tiles.
constexpr int64_t kSmallArea64 = 640 * 640, kSmallArea32 = 768 * 768;
constexpr int64_t kSmallMaxK = 1536;

// Tile choice by measured throughput on gfx950 at N = 8192: FP64 runs best
// with 8 waves of 64x32 and a 16-deep k-slab (71.7 TFLOP/s), FP32 with the
// 256x128 tile (140.6 TFLOP/s).  Smaller problems drop to smaller tiles while
// the larger ones would leave CUs idle (256 CUs).
GemmPlan plan_gemm(Elem e, int64_t M, int64_t N) {
  auto tiles = [&](int bm, int bn) { return (int)(((M + bm - 1) / bm) * ((N + bn - 1) / bn)); };
  GemmPlan p;
  if (!tile_override(&p.tile)) {
    if (e == Elem::F32 && tiles(256, 128) >= 256) p.tile = Tile::T256;
    else if (tiles(128, 128) >= 256) p.tile = Tile::T128W8;
    else if (M * N <= (e == Elem::F64 ? kSmallArea64 : kSmallArea32)) p.tile = Tile::T16;
    else if (tiles(64, 64) >= 128) p.tile = Tile::T64;
    else p.tile = Tile::T32;
  }
  const TileShape sh = shape_of(p.tile);
  p.tiles_m = (int)((M + sh.bm - 1) / sh.bm);
  p.tiles_n = (int)((N + sh.bn - 1) / sh.bn);
  return p;
}

int slab_of(Tile t) {
  return (t == Tile::T128K8 || t == Tile::T128W8K8 || t == Tile::T256K8) ? 8 : 16;
}

GemmPlan plan_gemm_k(Elem e, int64_t M, int64_t N, int64_t K) {
  GemmPlan p = plan_gemm(e, M, N);
  if (p.tile == Tile::T16) {
    if (K <= kSmallMaxK || getenv("NN_GEMM_TILE")) return p;  // four waves per tile over k
    // a long k extent: the split tiles
    auto tiles = [&](int bm, int bn) { return (int)(((M + bm - 1) / bm) * ((N + bn - 1) / bn)); };
    p.tile = tiles(64, 64) >= 128 ? Tile::T64 : Tile::T32;
    const TileShape sh = shape_of(p.tile);
    p.tiles_m = (int)((M + sh.bm - 1) / sh.bm);
    p.tiles_n = (int)((N + sh.bn - 1) / sh.bn);
  }
  const int64_t slabs = (K + slab_of(p.tile) - 1) / slab_of(p.tile);
  const char* v = getenv("NN_GEMM_SPLIT");
  int s = 1;
  if (v) {
    s = atoi(v);
    if (s < 1) s = 1;
    while (s > 1 && s > slabs) s >>= 1;
  } else {
    // aim at >= 1024 workgroups, each split keeping >= 32 slabs
    while (p.num_tiles() < 512 && (int64_t)p.num_tiles() * s * 2 <= 1024 && slabs / (s * 2) >= 32)
      s *= 2;
  }
  p.split = s;
  return p;
}

size_t gemm_work_bytes(const GemmPlan& plan, Elem e, int64_t M, int64_t N) {
  if (plan.split <= 1) return 0;
  // split partial products, then one sum of squares per tile row band
  return (size_t)plan.split * (size_t)M * (size_t)N * (e == Elem::F64 ? 8 : 4) +
         sizeof(double) * (size_t)plan.num_tiles() * kSplitChunks;
}

hipError_t launch_gemm(Elem e, bool cplx, const GemmPlan& plan, const GemmArgs& a,
                       hipStream_t s) {
  const bool al = aligned16(a.A) && aligned16(a.B);
  auto fits = [&](int v) {
    return al && a.lda % v == 0 && a.ldb % v == 0 && a.K % v == 0 && a.N % v == 0;
  };
  if (e == Elem::F64) {
    // complex: 16-byte elements, so K, N, lda, ldb (real) are always even
    if (cplx) return launch_tile<double, 2, true>(plan, a, s);
    return fits(2) ? launch_tile<double, 2, false>(plan, a, s)
                   : launch_tile<double, 1, false>(plan, a, s);
  }
  if (e == Elem::F32) {
    if (cplx)
      return fits(4) ? launch_tile<float, 4, true>(plan, a, s)
                     : launch_tile<float, 2, true>(plan, a, s);
    return fits(4) ? launch_tile<float, 4, false>(plan, a, s)
                   : launch_tile<float, 1, false>(plan, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace nn
