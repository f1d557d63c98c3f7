// nn_gemm_bf16.hip — BF16-input MFMA GEMM with FP32 accumulation (gfx950),
// used by the early nests of the mixed-precision schedule.
//
//   C = alpha * A * Bt^T + E + diag * I
//
// A (M x K) and Bt (N x K) are BF16, row-major, so both operands are read as
// runs of consecutive k (the right factor is handed over already transposed;
// the epilogue of the previous product writes that transposed copy).  The
// accumulator and E are FP32.  The epilogue can write any of: C in FP32, C in
// BF16 (row-major) and C^T in BF16, plus one FP64 sum of |C_ij|^2 per tile.
// BF16 rounding is round-to-nearest-even.
//
// MFMA: v_mfma_f32_16x16x32_bf16.  Lane l supplies A[l%16][8(l/16) .. +7] and
// Bt[l%16][8(l/16) .. +7] (16 bytes each) and returns rows 4 (l/16) + t of
// column l%16 (measured on gfx950).  Tile 128 x 128 x 64, 4 waves of 64 x 64,
// two LDS buffers, XCD-aware tile order as in the FP64/FP32 kernel.
#include <stdlib.h>

#include "nn_internal.h"

namespace nn {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 64, NT = 256;
constexpr int LDS_STRIDE = BK + 8;  // bf16 elements; 144-byte rows: conflict-free 16-byte reads

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __attribute__((aligned(16))) const unsigned int kZeroBf16[4] = {0u, 0u, 0u, 0u};

// Global loads through an address-space-1 pointer (a select between the
// matrix and kZeroBf16 otherwise becomes a flat load, which the LDS wait
// counter also tracks).
__device__ __forceinline__ u4_t load_global(uintptr_t addr) {
  return *reinterpret_cast<const __attribute__((address_space(1))) u4_t*>(addr);
}

__device__ __forceinline__ int xcd_remap(int bid, int nwg) {
  const int q = nwg / kNumXcd, r = nwg % kNumXcd;
  const int x = bid % kNumXcd, local = bid / kNumXcd;
  return x * q + (x < r ? x : r) + local;
}

// EXACT: M, N multiples of 128 and K of 64 (no bounds checks anywhere).
template <bool EXACT>
__global__ void __launch_bounds__(NT) gemm_bf16_kernel(Bf16GemmArgs p, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDS_STRIDE];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDS_STRIDE];
  __shared__ double red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tile order: XCD-contiguous ranges, 8 tile-rows per group
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int group = 8 * tiles_n;
  const int gid = tile / group, first = gid * 8;
  const int gsize = (tiles_m - first) < 8 ? (tiles_m - first) : 8;
  const int in = tile - gid * group;
  const int pm = first + in % gsize, pn = in / gsize;
  const int64_t m0 = (int64_t)pm * BM, n0 = (int64_t)pn * BN;
  const uint16_t* __restrict__ A = p.A;
  const uint16_t* __restrict__ Bt = p.Bt;

  f4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4_t{};

  // 128 rows x 64 k per operand and slab = 1024 16-byte vectors, 4 per thread
  u4_t ra[4], rb[4];
  const uintptr_t zaddr = reinterpret_cast<uintptr_t>(kZeroBf16);
  // exact tiling: wave-uniform slab base plus a fixed 32-bit offset per load
  const int r0 = tid >> 3, c0 = (tid & 7) * 8;  // row r0 + 32 i of the slab
  const uint32_t oa = (uint32_t)(r0 * p.lda + c0), ob = (uint32_t)(r0 * p.ldb + c0);
  const uint32_t sa32 = (uint32_t)(32 * p.lda), sb32 = (uint32_t)(32 * p.ldb);
  auto gload = [&](int64_t k0) {
    if constexpr (EXACT) {
      const uint16_t* a0 = A + m0 * p.lda + k0;
      const uint16_t* b0 = Bt + n0 * p.ldb + k0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ra[i] = load_global(reinterpret_cast<uintptr_t>(a0 + (oa + i * sa32)));
        rb[i] = load_global(reinterpret_cast<uintptr_t>(b0 + (ob + i * sb32)));
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = tid + i * NT;
        const int r = v >> 3, c = (v & 7) * 8;
        const int64_t gk = k0 + c;
        const int64_t ga = m0 + r, gb = n0 + r;
        const uintptr_t sa = reinterpret_cast<uintptr_t>(A + ga * p.lda + gk);
        const uintptr_t sb = reinterpret_cast<uintptr_t>(Bt + gb * p.ldb + gk);
        ra[i] = load_global((ga < p.M && gk < p.K) ? sa : zaddr);
        rb[i] = load_global((gb < p.N && gk < p.K) ? sb : zaddr);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int v = tid + i * NT;
      const int r = v >> 3, c = (v & 7) * 8;
      *reinterpret_cast<u4_t*>(&As[buf][r * LDS_STRIDE + c]) = ra[i];
      *reinterpret_cast<u4_t*>(&Bs[buf][r * LDS_STRIDE + c]) = rb[i];
    }
  };
  const int lr = lane & 15, lk = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      bf16x8_t af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const u4_t x = *reinterpret_cast<const u4_t*>(
            &As[buf][(wm * 64 + i * 16 + lr) * LDS_STRIDE + kk * 32 + 8 * lk]);
        af[i] = __builtin_bit_cast(bf16x8_t, x);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const u4_t x = *reinterpret_cast<const u4_t*>(
            &Bs[buf][(wn * 64 + j * 16 + lr) * LDS_STRIDE + kk * 32 + 8 * lk]);
        bf[j] = __builtin_bit_cast(bf16x8_t, x);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  };

  const int nk = (int)((p.K + BK - 1) / BK);
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk - 1; ++kt) {
    gload((int64_t)(kt + 1) * BK);
    // issue the global loads first and keep the LDS stores after all MFMAs
    __builtin_amdgcn_sched_barrier(0);
    compute(kt & 1);
    __builtin_amdgcn_sched_barrier(0);
    sstore((kt + 1) & 1);
    __syncthreads();
  }
  compute((nk - 1) & 1);

  double ss = 0.0;
  const float alpha = (float)p.alpha, diag = (float)p.diag;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = n0 + wn * 64 + j * 16 + lr;
      uint16_t tb[4];
      const int64_t rbase = m0 + wm * 64 + i * 16 + 4 * lk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t r = rbase + t;
        float v = 0.f;
        if (EXACT || (r < p.M && c < p.N)) {
          v = alpha * acc[i][j][t];
          if (p.E) v += p.E[r * p.lde + c];
          if (r == c) v += diag;
          if (p.C) p.C[r * p.ldc + c] = v;
          if (p.Cbf) p.Cbf[r * p.ldcb + c] = to_bf16(v);
          ss += (double)v * (double)v;
        }
        tb[t] = to_bf16(v);
      }
      if (p.CbfT && (EXACT || c < p.N)) {
        // C^T[c][rbase .. rbase + 3]: four consecutive bf16 of one transposed row
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (EXACT || rbase + t < p.M) p.CbfT[c * p.ldct + rbase + t] = tb[t];
      }
    }
  }
  if (p.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) p.partials[pm * tiles_n + pn] = red[0] + red[1] + red[2] + red[3];
  }
}

// Element-wise FP32/FP64 -> BF16 (and optionally the transposed copy) through
// a 32 x 32 LDS tile.
template <typename S>
__global__ void __launch_bounds__(256) cast_bf16_kernel(const S* src, int64_t lds, uint16_t* dst,
                                                        int64_t ldd, uint16_t* dstT, int64_t ldt,
                                                        int64_t rows, int64_t cols) {
  __shared__ uint16_t tile[32][33];
  const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = by + k, c = bx + tx;
    if (r < rows && c < cols) {
      const uint16_t b = to_bf16((float)src[r * lds + c]);
      if (dst) dst[r * ldd + c] = b;
      tile[k][tx] = b;
    }
  }
  if (!dstT) return;
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = bx + k, c = by + tx;  // dstT[r][c] = src[c][r]
    if (r < cols && c < rows) dstT[r * ldt + c] = tile[tx][k];
  }
}

}  // namespace

GemmPlan plan_gemm_bf16(int64_t M, int64_t N) {
  GemmPlan p;
  p.tile = Tile::T128;
  p.tiles_m = (int)((M + BM - 1) / BM);
  p.tiles_n = (int)((N + BN - 1) / BN);
  return p;
}

hipError_t launch_gemm_bf16(const GemmPlan& plan, const Bf16GemmArgs& a, hipStream_t s) {
  const int grid = plan.num_tiles();
  if (grid <= 0) return hipSuccess;
  if (a.M % BM == 0 && a.N % BN == 0 && a.K % BK == 0)
    hipLaunchKernelGGL(gemm_bf16_kernel<true>, dim3(grid), dim3(NT), 0, s, a, plan.tiles_m,
                       plan.tiles_n);
  else
    hipLaunchKernelGGL(gemm_bf16_kernel<false>, dim3(grid), dim3(NT), 0, s, a, plan.tiles_m,
                       plan.tiles_n);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(bool f64, const void* src, int64_t lds, uint16_t* dst, int64_t ldd,
                            uint16_t* dstT, int64_t ldt, int64_t rows, int64_t cols,
                            hipStream_t s) {
  const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  if (f64)
    hipLaunchKernelGGL((cast_bf16_kernel<double>), grid, dim3(256), 0, s,
                       static_cast<const double*>(src), lds, dst, ldd, dstT, ldt, rows, cols);
  else
    hipLaunchKernelGGL((cast_bf16_kernel<float>), grid, dim3(256), 0, s,
                       static_cast<const float*>(src), lds, dst, ldd, dstT, ldt, rows, cols);
  return hipGetLastError();
}

}  // namespace nn
