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
// column l%16 (measured on gfx950).  Two tilings: 128 x 128 x 64 with 4 waves
// of 64 x 64 (any shape), and 256 x 256 x 64 with 8 waves of 128 x 64 for large
// products (a wave reads 8 + 4 fragments for 32 MFMAs instead of 4 + 4 for 16).
// Both use two LDS buffers and the XCD-aware tile order of the FP64/FP32
// kernel.  LDS rows are 128 bytes (64 k) with the 16-byte segment s of row r
// stored at s ^ (r & 7), so the eight rows of a fragment read hit distinct
// banks (padded rows conflicted on gfx950).  For exact tilings the operands
// are loaded straight into LDS (global_load_lds_dwordx4: lane l of a wave
// writes bytes 16 l .. 16 l + 15 of a 1 KB block, measured on gfx950), which
// frees the staging registers and the LDS store instructions; other shapes
// stage through registers into the same layout.  Every output element
// is accumulated over the same k in the same order by the same instruction in
// all forms, so C is the same bits; only the per-tile partials differ.
#include <stdlib.h>

#include "nn_internal.h"

namespace nn {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

constexpr int BK = 64;

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

// Tile TBM x TBN x 64 over WGM x WGN waves.  EXACT: M, N multiples of the
// tile and K of 64 (no bounds checks anywhere).  DMA (exact tilings only):
// the operands go from global memory straight into LDS, 16 bytes per lane
// (global_load_lds_dwordx4), instead of through registers; see the loop.
template <int TBM, int TBN, int WGM, int WGN, bool EXACT, bool DMA = false>
__global__ void __launch_bounds__(64 * WGM * WGN)
    gemm_bf16_kernel(Bf16GemmArgs p, int tiles_m, int tiles_n) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int FI = TBM / WGM / 16, FJ = TBN / WGN / 16;  // 16 x 16 blocks per wave
  constexpr int VA = TBM * BK / 8 / NT, VB = TBN * BK / 8 / NT;  // 16-byte vectors per thread
  constexpr int RS = NT / 8;  // slab rows per staging pass
  static_assert(VA * NT * 8 == TBM * BK && VB * NT * 8 == TBN * BK, "staging must tile the slab");
  static_assert(!DMA || (EXACT && TBM % (8 * NW) == 0 && TBN % (8 * NW) == 0), "DMA form: exact");
  __shared__ double red[NW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  // tile order: XCD-contiguous ranges, 8 tile-rows per group
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int group = 8 * tiles_n;
  const int gid = tile / group, first = gid * 8;
  const int gsize = (tiles_m - first) < 8 ? (tiles_m - first) : 8;
  const int in = tile - gid * group;
  const int pm = first + in % gsize, pn = in / gsize;
  const int64_t m0 = (int64_t)pm * TBM, n0 = (int64_t)pn * TBN;
  const uint16_t* __restrict__ A = p.A;
  const uint16_t* __restrict__ Bt = p.Bt;

  f4_t acc[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) acc[i][j] = f4_t{};

  const int lr = lane & 15, lk = lane >> 4;
  if constexpr (DMA) {
    // LDS: per buffer and operand 256 rows x 64 k in 128-byte rows, no
    // padding (the load writes 64 lanes x 16 bytes = 1 KB contiguous per
    // instruction); 16-byte segment s of row r sits at segment s ^ (r & 7),
    // so the eight lanes of a fragment read (rows r..r+7, one segment) hit
    // eight distinct bank groups.
    __shared__ __attribute__((aligned(1024))) uint16_t Ad[2][TBM * BK];
    __shared__ __attribute__((aligned(1024))) uint16_t Bd[2][TBN * BK];
    // load instruction i of wave w covers slab rows DR i + 8 w .. + 7 (DR =
    // 8 NW rows per round); lane l fills row DR i + 8 w + l / 8, segment l % 8,
    // with global segment (l % 8) ^ (l / 8)
    constexpr int DR = 8 * NW;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int lrow = lane >> 3, gseg = (lane & 7) ^ lrow;
    const uint32_t oa = (uint32_t)((8 * wv + lrow) * p.lda + 8 * gseg);
    const uint32_t ob = (uint32_t)((8 * wv + lrow) * p.ldb + 8 * gseg);
    const uint32_t sar = (uint32_t)(DR * p.lda), sbr = (uint32_t)(DR * p.ldb);
    auto dma = [&](int buf, int64_t k0) {
      const uint16_t* a0 = A + m0 * p.lda + k0;
      const uint16_t* b0 = Bt + n0 * p.ldb + k0;
#pragma unroll
      for (int i = 0; i < TBM / DR; ++i)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(a0 + (oa + i * sar)),
            (__attribute__((address_space(3))) void*)(&Ad[buf][(DR * i + 8 * wv) * BK]),
            16, 0, 0);
#pragma unroll
      for (int i = 0; i < TBN / DR; ++i)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(b0 + (ob + i * sbr)),
            (__attribute__((address_space(3))) void*)(&Bd[buf][(DR * i + 8 * wv) * BK]),
            16, 0, 0);
    };
    // fragment (row R, k segment g) at R * 64 + 8 (g ^ (R & 7)); R & 7 = lr & 7
    const int arow = (wm * (16 * FI) + lr) * BK, brow = (wn * (16 * FJ) + lr) * BK;
    const int seg0 = 8 * ((0 * 4 + lk) ^ (lr & 7)), seg1 = 8 * ((1 * 4 + lk) ^ (lr & 7));
    const int nk = (int)(p.K / BK);
    dma(0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      bf16x8_t af[2][FI], bf[2][FJ];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int sg = kk ? seg1 : seg0;
#pragma unroll
        for (int i = 0; i < FI; ++i)
          af[kk][i] = __builtin_bit_cast(
              bf16x8_t, *reinterpret_cast<const u4_t*>(&Ad[buf][arow + i * 16 * BK + sg]));
#pragma unroll
        for (int j = 0; j < FJ; ++j)
          bf[kk][j] = __builtin_bit_cast(
              bf16x8_t, *reinterpret_cast<const u4_t*>(&Bd[buf][brow + j * 16 * BK + sg]));
      }
      // the other buffer was last read before the previous barrier
      if (kt + 1 < nk) dma(buf ^ 1, (int64_t)(kt + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kk][i], bf[kk][j], acc[i][j], 0, 0, 0);
      // keep every MFMA ahead of the wait, so the loads land while they run
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's loads are in LDS
      __syncthreads();
    }
  } else {
    // the same swizzled 128-byte rows as above (padded rows conflict on gfx950)
    __shared__ __attribute__((aligned(16))) uint16_t As[2][TBM * BK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][TBN * BK];
    // TBM (TBN) rows x 64 k per operand and slab in 16-byte vectors, VA (VB) per thread
    u4_t ra[VA], rb[VB];
    const uintptr_t zaddr = reinterpret_cast<uintptr_t>(kZeroBf16);
    // exact tiling: wave-uniform slab base plus a fixed 32-bit offset per load
    const int r0 = tid >> 3, c0 = (tid & 7) * 8;  // row r0 + RS i of the slab
    const uint32_t oa = (uint32_t)(r0 * p.lda + c0), ob = (uint32_t)(r0 * p.ldb + c0);
    const uint32_t sa32 = (uint32_t)(RS * p.lda), sb32 = (uint32_t)(RS * p.ldb);
    auto gload = [&](int64_t k0) {
      if constexpr (EXACT) {
        const uint16_t* a0 = A + m0 * p.lda + k0;
        const uint16_t* b0 = Bt + n0 * p.ldb + k0;
#pragma unroll
        for (int i = 0; i < VA; ++i)
          ra[i] = load_global(reinterpret_cast<uintptr_t>(a0 + (oa + i * sa32)));
#pragma unroll
        for (int i = 0; i < VB; ++i)
          rb[i] = load_global(reinterpret_cast<uintptr_t>(b0 + (ob + i * sb32)));
      } else {
        const int64_t gk = k0 + c0;
#pragma unroll
        for (int i = 0; i < VA; ++i) {
          const int64_t ga = m0 + r0 + i * RS;
          const uintptr_t sa = reinterpret_cast<uintptr_t>(A + ga * p.lda + gk);
          ra[i] = load_global((ga < p.M && gk < p.K) ? sa : zaddr);
        }
#pragma unroll
        for (int i = 0; i < VB; ++i) {
          const int64_t gb = n0 + r0 + i * RS;
          const uintptr_t sb = reinterpret_cast<uintptr_t>(Bt + gb * p.ldb + gk);
          rb[i] = load_global((gb < p.N && gk < p.K) ? sb : zaddr);
        }
      }
    };
    // row R's global segment c0 / 8 goes to segment (c0 / 8) ^ (R & 7); R & 7 =
    // r0 & 7 for every i (RS is a multiple of 8)
    const int sseg = 8 * ((c0 >> 3) ^ (r0 & 7));
    auto sstore = [&](int buf) {
#pragma unroll
      for (int i = 0; i < VA; ++i)
        *reinterpret_cast<u4_t*>(&As[buf][(r0 + i * RS) * BK + sseg]) = ra[i];
#pragma unroll
      for (int i = 0; i < VB; ++i)
        *reinterpret_cast<u4_t*>(&Bs[buf][(r0 + i * RS) * BK + sseg]) = rb[i];
    };
    auto compute = [&](int buf) {
#pragma unroll
      for (int kk = 0; kk < BK / 32; ++kk) {
        bf16x8_t af[FI], bf[FJ];
        const int sg = 8 * ((kk * 4 + lk) ^ (lr & 7));  // rows of a fragment: R & 7 = lr & 7
#pragma unroll
        for (int i = 0; i < FI; ++i) {
          const u4_t x = *reinterpret_cast<const u4_t*>(
              &As[buf][(wm * (16 * FI) + i * 16 + lr) * BK + sg]);
          af[i] = __builtin_bit_cast(bf16x8_t, x);
        }
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
          const u4_t x = *reinterpret_cast<const u4_t*>(
              &Bs[buf][(wn * (16 * FJ) + j * 16 + lr) * BK + sg]);
          bf[j] = __builtin_bit_cast(bf16x8_t, x);
        }
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j)
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
  }

  double ss = 0.0;
  const float alpha = (float)p.alpha, diag = (float)p.diag;
#pragma unroll
  for (int i = 0; i < FI; ++i) {
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      const int64_t c = n0 + wn * (16 * FJ) + j * 16 + lr;
      uint16_t tb[4];
      const int64_t rbase = m0 + wm * (16 * FI) + i * 16 + 4 * lk;
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
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += red[w];
      p.partials[pm * tiles_n + pn] = t;
    }
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

// The 256 x 256 tiling when it still gives every CU a tile (>= 256 tiles),
// else 128 x 128.  NN_BF16_TILE=128 or 256 forces one (read at each call).
GemmPlan plan_gemm_bf16(int64_t M, int64_t N) {
  GemmPlan p;
  const int64_t big = ((M + 255) / 256) * ((N + 255) / 256);
  bool use_big = big >= 256;
  if (const char* v = getenv("NN_BF16_TILE")) {
    if (atoi(v) == 128) use_big = false;
    if (atoi(v) == 256) use_big = true;
  }
  p.tile = use_big ? Tile::T256 : Tile::T128;
  const int t = use_big ? 256 : 128;
  p.tiles_m = (int)((M + t - 1) / t);
  p.tiles_n = (int)((N + t - 1) / t);
  return p;
}

hipError_t launch_gemm_bf16(const GemmPlan& plan, const Bf16GemmArgs& a, hipStream_t s) {
  const int grid = plan.num_tiles();
  if (grid <= 0) return hipSuccess;
  const int tm = plan.tile == Tile::T256 ? 256 : 128;
  if ((a.M + tm - 1) / tm != plan.tiles_m || (a.N + tm - 1) / tm != plan.tiles_n)
    return hipErrorInvalidValue;  // the plan was made for another shape
  const bool exact = a.M % tm == 0 && a.N % tm == 0 && a.K % BK == 0;
  const char* v = getenv("NN_BF16_DMA");  // 0: stage through registers instead
  const bool dma = !(v && atoi(v) == 0);
  if (tm == 256) {
    if (exact && dma)
      hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 2, 4, true, true>), dim3(grid), dim3(512), 0,
                         s, a, plan.tiles_m, plan.tiles_n);
    else if (exact)
      hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 2, 4, true>), dim3(grid), dim3(512), 0, s, a,
                         plan.tiles_m, plan.tiles_n);
    else
      hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 2, 4, false>), dim3(grid), dim3(512), 0, s,
                         a, plan.tiles_m, plan.tiles_n);
  } else if (exact && dma) {
    hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 2, 2, true, true>), dim3(grid), dim3(256), 0,
                       s, a, plan.tiles_m, plan.tiles_n);
  } else if (exact) {
    hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 2, 2, true>), dim3(grid), dim3(256), 0, s, a,
                       plan.tiles_m, plan.tiles_n);
  } else {
    hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 2, 2, false>), dim3(grid), dim3(256), 0, s, a,
                       plan.tiles_m, plan.tiles_n);
  }
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
