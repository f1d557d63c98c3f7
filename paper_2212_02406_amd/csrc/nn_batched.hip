// nn_batched.hip — many small NN inversions in one persistent launch (gfx950).
//
// Workload: the massive-MIMO regularised Gram matrices G = H^H H + s^2 I that
// motivate the Chebyshev-Neumann discussion after Corollary 4 of the paper
// (arXiv 2212.02406): thousands of Hermitian PD matrices of uneven sizes
// (K <= 64), a fixed number of nests at depth d (Sec. II-D Theorem).
//
// Structure:
//  * plan kernel (one block): stable counting sort of the matrices by size,
//    largest first (longest-processing-time order), the split into "group"
//    matrices (a whole 8-wave workgroup each), "pairs" (fixed-nest mode, K up
//    to 32: two matrices of one size per workgroup, four waves each) and
//    "wave" matrices (K <= wave_max_k, one wave each, eight per work item),
//    and the reset of the work counter.
//  * persistent kernel: each workgroup pops work items from the counter
//    until the queue is empty (every wave reaches that exit).  A matrix's
//    iterate and residual live in LDS for all its nests (buffers X and R, plus
//    U for depth >= 3); the residual reads G straight from global memory (L2
//    after the first read), and U = R + R R overwrites R at depth 2.  Two
//    buffers instead of four halve the LDS of a K = 64 complex matrix to
//    68 KB, so two workgroups share a CU.
//  * every product is an LDS-to-register GEMM on v_mfma_f32_16x16x4_f32; a
//    complex product is the real product of the interleaved left factor with
//    the real 2K x 2K form of the right factor, expanded on read (row 2k is
//    row k of B, row 2k+1 is that row with (re, im) -> (-im, re)).  The whole
//    product stays in registers until the group barrier, so the output may
//    overwrite an input buffer (X' = X + X U is written over X).
//  * results depend only on the matrix: every output block is summed over k
//    in the same order whichever wave holds it, and sums of squares add the
//    blocks' sums in block order, so a matrix gives the same bits alone or in
//    any batch, on the whole-group, paired or one-wave path.
//  * two control modes: a fixed number of nests, or a tolerance mode in which
//    each matrix applies the stopping rules of the single-matrix path on the
//    device after every residual (its own tolerance and nest limit), so the
//    matrices of one launch stop independently.
#include <math.h>

#include "nn_internal.h"

namespace nn {
namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kMaxN = 64;
// Eight waves per workgroup: a "group" matrix is shared by all eight (a K = 64
// complex product is 32 output blocks, 4 per wave), a "wave" item holds
// eight matrices of one wave each.
constexpr int kStageBatch = 16;  // global loads in flight per thread when staging G
constexpr int kDenLanes = 4;    // lanes per row or column sum of the transpose start
constexpr int kThreads = 512;
constexpr int kWaves = 8;
constexpr int kMaxBlocks = 8;  // 16x16 output blocks per wave
// Fixed-nest matrices of K in (wave_max_k, kQuadMaxK] run in pairs, four
// waves each, so that a workgroup's eight waves carry two blocks each instead
// of one: the two matrices of a pair have the same size and control flow and
// meet the same workgroup barriers.
constexpr int kQuadWaves = 4;
constexpr int kQuadMaxK = 32;

struct BatchHdr {
  int32_t counter;
  int32_t n_large;
  int32_t n_small;
  int32_t n_items;
  int32_t bad;
  int32_t n_quad;  // matrices in pairs (an even count)
  int32_t pad[2];
};

// LDS layout of a K x K matrix: real columns padded to a multiple of 16 plus
// 4 (row stride ld, a multiple of 4 floats so 16-byte reads stay aligned;
// ld = 4 or 20 mod 32 makes the 8-lane groups of those reads hit distinct
// banks), rows padded to a multiple of 16.  The padding is zero, so the
// MFMA loop needs no masks.
__device__ __host__ __forceinline__ int pad16(int x) { return (x + 15) & ~15; }
__device__ __host__ __forceinline__ int lds_ld(int K, bool cplx) {
  return pad16(cplx ? 2 * K : K) + 4;
}
__device__ __host__ __forceinline__ int lds_buf(int K, bool cplx) {
  return pad16(K) * lds_ld(K, cplx);
}

// Column swizzle of complex rows: when a row's padded width is a multiple of
// 32 floats, rows 2 and 3 mod 4 store column c at c ^ 16.  With ld = 4 mod 32
// the B-fragment reads of a k-group (complex rows 2 lk and 2 lk + 1 for lane
// quarter lk) otherwise put lane quarters 0 and 1 on overlapping banks (row
// offset 2 ld = 8 mod 64); the swizzle moves one of them 16 banks away.
// 16-byte segments stay whole (bit 4 only) and the A-fragment reads stay
// conflict free.  swz: 0 or 16.
__device__ __host__ __forceinline__ int lds_swz(int K, bool cplx) {
  return cplx && (pad16(2 * K) & 31) == 0 ? 16 : 0;
}
__device__ __forceinline__ int scol(int r, int c, int swz) { return c ^ (((r >> 1) & 1) * swz); }

// Dynamic LDS of the persistent kernel (matrix buffers) and the per-group
// reduction scratch.  Everything below addresses LDS through these arrays and
// integer offsets, so the accesses compile to ds_read/ds_write.
extern __shared__ __attribute__((aligned(16))) float smem[];
__shared__ double s_red[kWaves][8 + 2 * kMaxN];

struct Group {
  int gw;      // wave index inside the group
  int G;       // waves in the group (4 or 1)
  int lane;
  int gtid;    // thread index inside the group
  int redrow;  // row of s_red this group uses
  bool whole;  // the group is the whole workgroup
  __device__ __forceinline__ void sync() const {
    if (whole) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

typedef float f2_t __attribute__((ext_vector_type(2)));

// Operands of one k-group (16 real k) for NB output blocks.  SH: the NB
// blocks of a wave lie in one block row and share their A fragment.
template <bool CPLX, int NB, bool SH>
struct KFrag {
  f4_t a[SH ? 1 : NB];
  f4_t b[NB];  // complex: this lane's column of two complex rows (x, y); real: 4 rows
};

template <bool CPLX, int NB, bool SH, bool WITH_A = true>
__device__ __forceinline__ void load_kgroup(KFrag<CPLX, NB, SH>& f, const int* aoff,
                                            const int* boff, int j, int ld, int sa) {
  if constexpr (WITH_A) {
#pragma unroll
    for (int i = 0; i < (SH ? 1 : NB); ++i)
      f.a[i] = *static_cast<const f4_t*>(
          __builtin_assume_aligned(&smem[aoff[i] + ((16 * j) ^ sa)], 16));
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (CPLX) {
      const int o = boff[i] + 8 * j * ld;
      f.b[i] = f4_t{smem[o], smem[o + ld], 0.f, 0.f};
    } else {
      const int o = boff[i] + 16 * j * ld;
      f.b[i] = f4_t{smem[o], smem[o + ld], smem[o + 2 * ld], smem[o + 3 * ld]};
    }
  }
}

// The four MFMA steps of a k-group, step-major over the blocks: consecutive
// MFMAs write different accumulators, so one does not wait for the previous
// one's result (each accumulator still sums its k in the same order).
// The value lane n ^ 1 holds (adjacent lanes swap: DPP quad_perm 1,0,3,2).
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}

template <bool CPLX, int NB, bool SH>
__device__ __forceinline__ void mma_kgroup(f4_t* acc, const KFrag<CPLX, NB, SH>& f,
                                           const int* sgn) {
  float b[NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (CPLX) {
      // expanded rows 2 kc and 2 kc + 1 of the complex rows kc0, kc0 + 1 at
      // this lane's real column n: row 2 kc is B[kc][n] as stored; row 2 kc + 1
      // is -B[kc][n + 1] for even n (-im) and B[kc][n - 1] for odd n (re),
      // i.e. the partner lane's value with the sign bit flipped on even lanes
      b[i][0] = f.b[i].x;
      b[i][1] = __int_as_float(__float_as_int(pair_swap(f.b[i].x)) ^ sgn[i]);
      b[i][2] = f.b[i].y;
      b[i][3] = __int_as_float(__float_as_int(pair_swap(f.b[i].y)) ^ sgn[i]);
    } else {
      b[i][0] = f.b[i].x;
      b[i][1] = f.b[i].y;
      b[i][2] = f.b[i].z;
      b[i][3] = f.b[i].w;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < NB; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[SH ? 0 : i][q], b[i][q], acc[i], 0, 0, 0);
}

// C = alpha * A B + E + diag * I on K x K matrices held in LDS at float
// offsets A, B, E (E < 0: none), C, row stride ld, zero padding as above.
// C may alias A, B or E.  If ss is non-null the group's sum of |C_ij|^2 is
// returned through it.  NB = blocks per wave, the same for every wave of the
// group; a wave's blocks past the last one recompute that block and do not
// store it.
//
// k-assignment: in k-group j (16 real k) MFMA step q takes, for the lanes of
// quarter lk, k = 16 j + 4 lk + q.  Each step still covers four distinct k, and
// a lane's four A values of the group are contiguous (one 16-byte read).  For
// a complex B the four k are the rows 2 kc, 2 kc + 1 of two complex rows: a
// lane reads its own column of each complex row and takes the other half of
// the (re, im) pair from the adjacent lane (DPP), so the expansion costs two
// 4-byte reads and two lane swaps per block and k-group.  All operand reads
// of a k-group are issued before its MFMAs; when a wave's blocks share a block
// row (SH) their A fragment is read once.  (Reading k-group j + 1 during the
// MFMAs of k-group j needs a second register set, which made the compiler
// spill in this fully inlined kernel.)
//
// GA: the left factor is read from global memory instead of LDS (Ag, row-major
// K x cols floats); the residual R = I - G X reads G this way, so G is staged
// into LDS only once, for the transpose start, not before every residual.  A lane's fragment of k-group j + 1 is loaded while the MFMAs of
// k-group j run (L2 latency hidden by one k-group); out-of-range fragments
// read as zero, as the LDS padding does, so both forms give the same bits.
template <bool CPLX, int NB, bool SH, bool GA = false>
__device__ __forceinline__ void lds_gemm_nb(int A, int B, int E, int C, int K, int ld,
                                            float alpha, float diag, const Group& g,
                                            double* ss, int swz, const float* Ag = nullptr) {
  const int cols = CPLX ? 2 * K : K;
  const int nbm = (K + 15) >> 4, nbn = (cols + 15) >> 4, nb = nbm * nbn;
  const int first = g.gw * NB;
  const int lr = g.lane & 15, lk = g.lane >> 4;
  // swizzle of this lane's A rows (bm 16 + lr) and B rows (complex 8 j + 2 lk
  // and + 1): fixed per lane
  const int sa = ((lr >> 1) & 1) * swz, sb = (lk & 1) * swz;
  f4_t acc[NB];
  int aoff[NB], boff[NB], bm_[NB], bn_[NB], sgn[NB];
  bool live[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    acc[i] = f4_t{};
    live[i] = first + i < nb;
    const int b = live[i] ? first + i : nb - 1;
    bm_[i] = b / nbn;
    bn_[i] = b - bm_[i] * nbn;
    const int n = bn_[i] * 16 + lr;
    aoff[i] = A + (bm_[i] * 16 + lr) * ld + 4 * lk;
    if constexpr (CPLX) {
      boff[i] = B + (2 * lk) * ld + (n ^ sb);
      sgn[i] = (n & 1) ? 0 : (int)0x80000000u;
    } else {
      boff[i] = B + (4 * lk) * ld + n;
      sgn[i] = 0;
    }
  }
  const int kgroups = nbn;  // padded real inner dimension / 16
  // A wave issues each k-group's MFMAs at raised priority (s_setprio 1), so
  // the burst is not interleaved with the other waves' operand reads and
  // epilogues (K = 64 batch, depth 2: 2-5% less time per nest; the opposite
  // choice, the reads at raised priority, made the nest times erratic).
  if constexpr (GA) {
    constexpr int NA = SH ? 1 : NB;
    const float* arow[NA];
    bool aok[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int m = bm_[i] * 16 + lr;
      aok[i] = m < K;
      arow[i] = Ag + (aok[i] ? m : 0) * cols + 4 * lk;
    }
    // 16-byte loads when every row starts 16-byte aligned, else four 4-byte
    // loads (uniform choice)
    const bool vec = (reinterpret_cast<uintptr_t>(Ag) & 15) == 0 && (cols & 3) == 0;
    auto gload = [&](int j, f4_t* dst) {
      const int c = 16 * j + 4 * lk;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        if (vec) {
          dst[i] = aok[i] && c < cols ? *reinterpret_cast<const f4_t*>(arow[i] + 16 * j)
                                      : f4_t{};
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) dst[i][e] = aok[i] && c + e < cols ? arow[i][16 * j + e] : 0.f;
        }
      }
    };
    f4_t an[NA];
    gload(0, an);
    for (int j = 0; j < kgroups; ++j) {
      KFrag<CPLX, NB, SH> f;
#pragma unroll
      for (int i = 0; i < NA; ++i) f.a[i] = an[i];
      if (j + 1 < kgroups) gload(j + 1, an);
      load_kgroup<CPLX, NB, SH, false>(f, aoff, boff, j, ld, sa);  // B only
      __builtin_amdgcn_s_setprio(1);
      mma_kgroup<CPLX, NB, SH>(acc, f, sgn);
      __builtin_amdgcn_s_setprio(0);
    }
  } else {
    for (int j = 0; j < kgroups; ++j) {
      KFrag<CPLX, NB, SH> f;
      load_kgroup<CPLX, NB, SH>(f, aoff, boff, j, ld, sa);  // all operand reads of the group first
      __builtin_amdgcn_s_setprio(1);
      mma_kgroup<CPLX, NB, SH>(acc, f, sgn);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  // Epilogue in registers (rows 4 (lane/16) + t of each block, FP32 layout).
  // Every E read is issued before the first use.  Entries outside a ragged
  // matrix lie in the zero padding of the buffers and are set to zero here, so
  // the padding stays zero and the stores need no per-element test.
  float ev[NB][4];
  if (E >= 0) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int n = bn_[i] * 16 + lr;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = bm_[i] * 16 + 4 * lk + t;
        ev[i][t] = smem[E + m * ld + scol(m, n, swz)];
      }
    }
  }
  double ssq[NB];  // this lane's part of each block's sum of squares
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int n = bn_[i] * 16 + lr;
    ssq[i] = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int m = bm_[i] * 16 + 4 * lk + t;
      float v = alpha * acc[i][t];
      if (E >= 0) v += ev[i][t];
      if (CPLX ? (n == 2 * m) : (n == m)) v += diag;
      v = m < K && n < cols ? v : 0.f;
      acc[i][t] = v;
      if (ss) ssq[i] += (double)v * (double)v;
    }
  }
  // every read of A, B, E is done before C (which may alias them) is written;
  // the residual's C aliases none of its LDS inputs
  if (C == B || C == E || (!GA && C == A)) g.sync();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (!live[i]) continue;  // a recomputed copy of another wave's block
    const int n = bn_[i] * 16 + lr;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int m = bm_[i] * 16 + 4 * lk + t;
      smem[C + m * ld + scol(m, n, swz)] = acc[i][t];
    }
  }
  if (ss) {
    // Each block's sum (a butterfly over the lanes), then the blocks in block
    // order: the same association whichever waves hold the blocks, so a
    // matrix's rms has the same bits on the whole-group, paired and one-wave
    // paths (and in both control modes).
#pragma unroll
    for (int i = 0; i < NB; ++i) ssq[i] = wave_sum(ssq[i]);
    if (g.lane == 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (live[i]) s_red[g.redrow][first + i] = ssq[i];
    }
    g.sync();
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += s_red[g.redrow][b];
    *ss = t;
  }
  g.sync();
}

// Blocks per wave for a K x K product over G waves, rounded up to 1, 2, 4 or
// 8 (the kernel is instantiated for those counts only).
__device__ __host__ __forceinline__ int blocks_per_wave(int K, bool cplx, int G) {
  const int cols = cplx ? 2 * K : K;
  const int nb = ((K + 15) >> 4) * ((cols + 15) >> 4);
  const int per = (nb + G - 1) / G;
  return per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : 8;
}

// Whether the NB blocks of each wave lie in one block row (NB divides the
// number of column blocks), so they can share one A fragment per k-group.
__device__ __forceinline__ bool shared_rows(int K, bool cplx, int NB) {
  const int nbn = ((cplx ? 2 * K : K) + 15) >> 4;
  return nbn % NB == 0;
}

// LDS buffers per matrix: X and R (R also holds the staged G and, at depth
// <= 2, U), plus U for depth >= 3.
__device__ __host__ __forceinline__ int lds_nbufs(int depth) { return depth >= 3 ? 3 : 2; }

// The whole NN run for one matrix: load, start iterate, then either `iters`
// nests and a final residual (iters > 0) or the tolerance-mode loop (iters ==
// 0): after each residual R_k = I - G X_k, in this order, rms_k not finite ->
// NONFINITE; rms_k < tol -> OK with X_k; k > 0, rms_k >= 1 and rising ->
// DIVERGED; k > 0, sqrt(K) rms_{k-1} < 0.1 and rms_k >= rms_{k-1} -> STAGNATED
// with X_{k-1}; k == max_iter -> NOT_CONVERGED; else one nest.  X_{k-1} is
// kept in global memory: X_k is written out before its nest whenever
// sqrt(K) rms_k < 0.1, the only case in which the next test can fire.  Every
// decision uses the group-reduced sum, identical in all lanes, so the group's
// control flow stays uniform.
template <bool CPLX, int NB, bool SH, bool TOL>
__device__ __forceinline__ void invert_one(const float* Ag, float* Xg, int K, int depth, int x0,
                                           int iters, double tol, int max_iter, int buf,
                                           int bufstride, const Group& g, nn_info_dev* info) {
  const int cols = CPLX ? 2 * K : K;
  const int ld = lds_ld(K, CPLX);
  const int swz = lds_swz(K, CPLX);
  const int Xs = buf, Rs = buf + bufstride, Us = depth >= 3 ? buf + 2 * bufstride : Rs;
  const int Gs = Rs;  // G is staged into R's buffer
  double* red = s_red[g.redrow];
  const int nthr = g.G * 64;
  if ((K & 15) || (cols & 15)) {  // ragged size: the padding must read as zero
    const int nb = lds_buf(K, CPLX);
    for (int q = 0; q < lds_nbufs(depth); ++q)
      for (int e = g.gtid; e < nb; e += nthr) smem[buf + q * bufstride + e] = 0.f;
  }
  // unconditional, so that how many barriers a matrix meets does not depend on
  // its size (the two matrices of a pair share the workgroup barriers)
  g.sync();
  // Staging of a row-major K x cols matrix into an LDS buffer: the group's
  // threads take consecutive elements (coalesced) and issue kStageBatch loads
  // before storing any, so a K = 64 complex matrix costs one memory round
  // trip per thread instead of one per element.  A thread's element
  // e = r cols + c advances by nthr = dr cols + dc per load, so (r, c) is
  // carried along without a division per element.
  auto stage = [&](int dst, const float* src) {
    const int tot = K * cols;
    const int dr = nthr / cols, dc = nthr - dr * cols;
    int r = g.gtid / cols, c = g.gtid - r * cols;
    for (int e0 = g.gtid; e0 < tot; e0 += kStageBatch * nthr) {
      float v[kStageBatch];
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        const int e = e0 + u * nthr;
        v[u] = e < tot ? src[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kStageBatch; ++u) {
        if (e0 + u * nthr < tot) smem[dst + r * ld + scol(r, c, swz)] = v[u];
        c += dc;
        r += dr;
        if (c >= cols) {
          c -= cols;
          ++r;
        }
      }
    }
  };
  auto stage_g = [&]() {
    stage(Gs, Ag);
    g.sync();
  };
  auto store_x = [&]() {
    for (int r = g.gw; r < K; r += g.G)
      for (int c = g.lane; c < cols; c += 64) Xg[r * cols + c] = smem[Xs + r * ld + scol(r, c, swz)];
  };
  // The transpose start reads G (rows and columns) from LDS: G is staged into
  // R's buffer once, with all of a thread's loads in flight.  The other starts
  // need only G's diagonal (read from global memory below) or nothing, and
  // the residuals read G from global memory anyway, so they skip the staging
  // (identity start, 4096-matrix batch: 0.394 -> 0.384 ms).
  if (x0 == NN_X0_TRANSPOSE) stage_g();
  else g.sync();
  // Start iterate (Sec. II-A normalisation): den = ||G||_1 ||G||_inf or Re Tr G;
  // NN_X0_GIVEN reads X_0 from Xg.
  double den = 1.0;
  if (x0 == NN_X0_TRANSPOSE) {
    // 2K sums of K moduli (rows 0..K-1, then columns), each split over
    // kDenLanes adjacent lanes (element j to lane j mod kDenLanes, then a
    // shuffle tree): the order depends on K only, not on the group size, so a
    // matrix gets the same den on the one-wave and the whole-group path.
    const int per_pass = nthr / kDenLanes;
    for (int base = 0; base < 2 * K; base += per_pass) {
      const int sidx = base + g.gtid / kDenLanes, part = g.gtid % kDenLanes;
      double s = 0.0;
      if (sidx < 2 * K) {
        const bool row = sidx < K;
        const int i = row ? sidx : sidx - K;
        for (int j = part; j < K; j += kDenLanes) {
          const int r = row ? i : j, c = row ? j : i;
          if constexpr (CPLX) {
            const double re = smem[Gs + r * ld + scol(r, 2 * c, swz)];
            const double im = smem[Gs + r * ld + scol(r, 2 * c + 1, swz)];
            s += sqrt(re * re + im * im);
          } else {
            s += fabs((double)smem[Gs + r * ld + c]);
          }
        }
      }
#pragma unroll
      for (int o = kDenLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (sidx < 2 * K && part == 0) red[8 + sidx] = s;
    }
    g.sync();
    // ||G||_inf = max over rows, ||G||_1 = max over columns: lane l takes row
    // and column l (K <= 64), then a wave maximum (every wave the same)
    const int l = g.lane;
    double ninf = l < K ? red[8 + l] : 0.0, n1 = l < K ? red[8 + K + l] : 0.0;
    int bad = !isfinite(ninf) || !isfinite(n1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double a = __shfl_xor(ninf, o, 64), b = __shfl_xor(n1, o, 64);
      ninf = a > ninf ? a : ninf;
      n1 = b > n1 ? b : n1;
      bad |= __shfl_xor(bad, o, 64);
    }
    den = bad ? NAN : n1 * ninf;
  } else if (x0 == NN_X0_SCALED_IDENTITY) {
    // lane i loads diagonal entry i (K <= 64); the entries are then added in
    // index order through readlane
    const float dg = g.lane < K ? Ag[g.lane * cols + (CPLX ? 2 * g.lane : g.lane)] : 0.f;
    double t = 0.0;
    for (int i = 0; i < K; ++i)
      t += (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(dg), i));
    den = t;
  }
  const bool den_ok = isfinite(den) && den > 0.0;
  const float s = (float)(1.0 / den);
  g.sync();
  if (x0 == NN_X0_GIVEN) {
    stage(Xs, Xg);
  } else {
    for (int r = g.gw; r < K; r += g.G) {
      for (int c = g.lane; c < cols; c += 64) {
        float v;
        if (x0 == NN_X0_TRANSPOSE) {
          if constexpr (CPLX) {
            const int j = c >> 1;  // X[r][j] = conj(G[j][r]) * s
            v = (c & 1) ? -smem[Gs + j * ld + scol(j, 2 * r + 1, swz)] * s
                        : smem[Gs + j * ld + scol(j, 2 * r, swz)] * s;
          } else {
            v = smem[Gs + c * ld + r] * s;
          }
        } else {
          v = (CPLX ? (c == 2 * r) : (c == r)) ? s : 0.f;
        }
        smem[Xs + r * ld + scol(r, c, swz)] = v;
      }
    }
  }
  g.sync();
  constexpr bool fixed = !TOL;  // TOL: iters == 0 (tolerance mode), else iters nests
  const double sqk = sqrt((double)K);
  int k = 0, status = NN_OK;
  double rms = NAN, rms_prev = NAN;
  bool use_prev = false;
  if (!fixed && !den_ok) {
    status = isfinite(den) ? NN_ERR_DIVERGED : NN_ERR_NONFINITE;
  } else {
    for (;;) {
      double ss = 0.0;
      const bool want = !fixed || k == iters;
      lds_gemm_nb<CPLX, NB, SH, true>(-1, Xs, -1, Rs, K, ld, -1.f, 1.f, g, want ? &ss : nullptr,
                                      swz, Ag);  // R = I - G X
      if (fixed) {
        if (k == iters) {
          rms = sqrt(ss / (double)K);
          status = !den_ok ? (isfinite(den) ? NN_ERR_DIVERGED : NN_ERR_NONFINITE)
                           : (isfinite(rms) ? NN_OK : NN_ERR_NONFINITE);
          break;
        }
      } else {
        rms = sqrt(ss / (double)K);
        if (!isfinite(rms)) {
          status = NN_ERR_NONFINITE;
          break;
        }
        if (rms < tol) break;
        if (k > 0 && rms >= 1.0 && rms > rms_prev) {
          status = NN_ERR_DIVERGED;
          break;
        }
        if (k > 0 && sqk * rms_prev < 0.1 && rms >= rms_prev) {
          status = NN_STAGNATED;
          use_prev = true;
          break;
        }
        if (k >= max_iter) {
          status = NN_NOT_CONVERGED;
          break;
        }
        if (sqk * rms < 0.1) store_x();  // X_k, in case the next nest stagnates
      }
      int U = Rs;
      for (int m = 1; m < depth; ++m) {  // U_{m+1} = R + R U_m
        lds_gemm_nb<CPLX, NB, SH>(Rs, U, Rs, Us, K, ld, 1.f, 0.f, g, nullptr, swz);
        U = Us;
      }
      lds_gemm_nb<CPLX, NB, SH>(Xs, U, Xs, Xs, K, ld, 1.f, 0.f, g, nullptr, swz);  // X = X + X U
      rms_prev = rms;
      ++k;
    }
  }
  if (!use_prev) store_x();
  if (info && g.gtid == 0) {
    nn_info_dev d;
    d.iters = use_prev ? k - 1 : k;
    d.rms = use_prev ? rms_prev : rms;
    d.status = status;
    *info = d;
  }
  g.sync();
}

// Plan of one launch: a stable counting sort of the matrices by size, largest
// first (longest-processing-time order), into four regions of perm:
//   large  K > quad_max_k, one matrix per 8-wave item, then one matrix of each
//          quad-class size with an odd count (also run as a whole item);
//   quad   wave_max_k < K <= quad_max_k, pairs of equal size, one pair per
//          item (four waves each);
//   small  K <= wave_max_k, eight matrices per item (one wave each);
// then the entries with an invalid size (reported, never run).  Within a size
// the order is the batch order: each wave ranks its lanes by ballots and the
// waves' counts are prefix-summed, so the plan is the same on every run.
__global__ void __launch_bounds__(1024) batched_plan(const int32_t* sizes, int batch, int max_n,
                                                     int wave_max_k, int quad_max_k,
                                                     BatchHdr* hdr, int32_t* perm,
                                                     nn_info_dev* info) {
  constexpr int NW = 1024 / 64;
  __shared__ int cnt[kMaxN + 1], start[kMaxN + 1], left[kMaxN + 1], coff[kMaxN + 1],
      ctot[kMaxN + 1];
  __shared__ int wcnt[NW][kMaxN + 1], wpre[NW][kMaxN + 1];
  __shared__ int bad;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  if (t <= kMaxN) {
    cnt[t] = 0;
    coff[t] = 0;
  }
  for (int e = t; e < NW * (kMaxN + 1); e += 1024) (&wcnt[0][0])[e] = 0;
  if (t == 0) bad = 0;
  __syncthreads();
  // size of entry b (0: invalid, reported), -1 past the end of the batch
  auto size_of = [&](int b) {
    if (b >= batch) return -1;
    const int k = sizes[b];
    return k < 1 || k > max_n ? 0 : k;
  };
  // The first kPlanRegs chunks' sizes are loaded once, all at the same time
  // (each pass over them would otherwise wait for one memory round trip per
  // chunk); later chunks are read as they come.
  constexpr int kPlanRegs = 8;
  int kreg[kPlanRegs];
#pragma unroll
  for (int i = 0; i < kPlanRegs; ++i) kreg[i] = size_of(i * 1024 + t);
  auto size_at = [&](int i) {
    int k = -1;
#pragma unroll
    for (int q = 0; q < kPlanRegs; ++q)
      if (q == i) k = kreg[q];
    return i < kPlanRegs ? k : size_of(i * 1024 + t);
  };
  // Calls fn(kk, m) once per size kk present in the wave (m: the lanes holding
  // it) and returns this lane's rank among the lanes with its size.
  auto per_size = [&](int k, auto fn) {
    int rank = 0;
    uint64_t todo = __ballot(k >= 0);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const int kk = __shfl(k, leader, 64);
      const uint64_t m = __ballot(k == kk);
      if (k == kk) rank = __popcll(m & ((1ull << lane) - 1));
      if (lane == leader) fn(kk, m);
      todo &= ~m;
    }
    return rank;
  };
  // counts (one atomic per wave and size present)
  for (int c0 = 0; c0 < batch; c0 += 1024) {
    const int k = size_at(c0 / 1024);
    if (k == 0) {
      bad = 1;
      if (info) {
        nn_info_dev d;
        d.iters = 0;
        d.status = NN_ERR_ARG;
        d.rms = NAN;
        info[c0 + t] = d;
      }
    }
    (void)per_size(k, [&](int kk, uint64_t m) { atomicAdd(&cnt[kk], (int)__popcll(m)); });
  }
  __syncthreads();
  const int wk = wave_max_k, qk = quad_max_k > wave_max_k ? quad_max_k : wave_max_k;
  static_assert(kMaxN == 64, "one lane per size");
  if (w == 0) {
    // the region offsets by 64-lane prefix sums, lane l holding size 64 - l
    // (sizes in descending order along the lanes)
    const int k = kMaxN - lane, c = cnt[k];
    auto scan = [&](int x, int* total) {  // exclusive prefix over the lanes
      int incl = x;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      *total = __shfl(incl, 63, 64);
      return incl - x;
    };
    const bool lg = k > qk, qd = k <= qk && k > wk;
    int n0, nl, nq, ns;
    const int a = scan(lg ? c : 0, &n0);                       // large, K descending
    const int b = scan(qd && (c & 1) ? 1 : 0, &nl);            // one odd one out per pair size
    const int q = scan(qd ? c & ~1 : 0, &nq);                  // pairs
    const int sm = scan(!lg && !qd ? c : 0, &ns);              // one wave per matrix
    const int n_large = n0 + nl;
    if (lg) start[k] = a;
    if (qd) {
      if (c & 1) left[k] = n0 + b;
      start[k] = n_large + q;
    }
    if (!lg && !qd) start[k] = n_large + nq + sm;
    if (lane == 0) {
      start[0] = n_large + nq + ns;
      hdr->counter = 0;
      hdr->n_large = n_large;
      hdr->n_quad = nq;
      hdr->n_small = ns;
      hdr->n_items = n_large + nq / 2 + (ns + kWaves - 1) / kWaves;
      hdr->bad = bad;
    }
  }
  __syncthreads();
  for (int c0 = 0; c0 < batch; c0 += 1024) {
    const int k = size_at(c0 / 1024);
    const int rank = per_size(k, [&](int kk, uint64_t m) { wcnt[w][kk] = (int)__popcll(m); });
    __syncthreads();
    // exclusive prefix of the waves' counts per size: 16-lane groups, one
    // size per group, one wave per lane
    for (int base = 0; base <= kMaxN; base += 1024 / NW) {
      const int kk = base + (t >> 4), v = t & (NW - 1);
      const int x = kk <= kMaxN ? wcnt[v][kk] : 0;
      int incl = x;
#pragma unroll
      for (int o = 1; o < NW; o <<= 1) {
        const int y = __shfl_up(incl, o, NW);
        if (v >= o) incl += y;
      }
      if (kk <= kMaxN) {
        wpre[v][kk] = incl - x;
        if (v == NW - 1) ctot[kk] = incl;
      }
    }
    __syncthreads();
    for (int e = t; e < NW * (kMaxN + 1); e += 1024) (&wcnt[0][0])[e] = 0;
    if (k >= 0) {
      const int r = coff[k] + wpre[w][k] + rank;  // rank among all entries of size k
      const bool odd_last = k > wk && k <= qk && (cnt[k] & 1) && r == cnt[k] - 1;
      perm[odd_last ? left[k] : start[k] + r] = c0 + t;
    }
    __syncthreads();
    if (t <= kMaxN) coff[t] += ctot[t];
  }
}

// waves_per_eu(4): at most 128 registers per lane (VGPRs and AGPRs), so two
// eight-wave workgroups (four waves per SIMD) share a CU; the fully inlined
// size-class paths otherwise take about 400 and hold a SIMD to one wave.
// Measured on 4096 K = 64 complex matrices: 2.53 ms (four waves per
// workgroup, ~400 registers), 1.84 ms (four waves, 256 registers, two
// workgroups per CU), 1.58 ms (eight waves, 128 registers, two per CU; about
// 1 KB of scratch spills per lane).  TOL selects the control mode at compile
// time (tolerance mode, a.iters == 0, or a fixed number of nests), so the
// fixed-nest kernel carries none of the per-nest stopping logic.
// MAXNB: the largest blocks-per-wave count compiled in (4 or 8).  The 8-block
// paths (one-wave complex matrices of K in 17..32, only reachable with a
// one-wave limit of 32) hold the most registers; compiling them only when a
// launch can reach them takes the other launches from 682 spilled registers
// per lane to about 120 (gfx950, 128-register budget).  The host picks the
// instantiation (batched_max_nb); an item that would need more blocks than
// compiled in is reported as unsupported rather than computed.
template <bool CPLX, bool TOL, int MAXNB>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
batched_nn(BatchedArgs a, const int32_t* perm, BatchHdr* hdr) {
  __shared__ int item_s;
  // Values that are the same for a whole wave (the work item, the matrix and
  // its size) are read through readfirstlane, so the compiler keeps them and
  // everything derived from them (strides, block counts, loop bounds) in
  // scalar registers and runs the k-loops as uniform loops.
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cm = CPLX ? 2 : 1;
  const float* A = static_cast<const float*>(a.A);
  float* X = static_cast<float*>(a.X);
  const int64_t* xoffsets = a.xoffsets ? a.xoffsets : a.offsets;
  const int big_stride = lds_buf(a.max_n, CPLX);
  const int wk = a.wave_max_k > 0 ? a.wave_max_k : 1;
  const int wave_stride = lds_buf(wk, CPLX);
  const int quad_stride = lds_buf(a.quad_max_k > 0 ? a.quad_max_k : 1, CPLX);
  const int n_items = hdr->n_items, n_large = hdr->n_large, n_small = hdr->n_small;
  const int n_quad = TOL ? 0 : hdr->n_quad;
  for (;;) {
    if (tid == 0) item_s = atomicAdd(&hdr->counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();
    if (item >= n_items) break;
    if (item < n_large) {
      const int b = __builtin_amdgcn_readfirstlane(perm[item]);
      const Group g{wave, kWaves, lane, tid, 0, true};
      const int64_t off = a.offsets[b] * cm, xoff = xoffsets[b] * cm;
      const int K = __builtin_amdgcn_readfirstlane(a.sizes[b]);
      const double tol = a.tols ? a.tols[b] : a.tol;
      const int mit = a.maxits ? a.maxits[b] : a.max_iter;
      nn_info_dev* inf = a.info ? a.info + b : nullptr;
      const int nbw = blocks_per_wave(K, CPLX, kWaves);
      const bool sh = shared_rows(K, CPLX, nbw);
#define NN_ONE(NB, SH)                                                                     \
  invert_one<CPLX, NB, SH, TOL>(A + off, X + xoff, K, a.depth, a.x0, a.iters, tol, mit, 0,   \
                                big_stride, g, inf)
      switch (nbw * 2 + (sh ? 1 : 0)) {
        case 2:
        case 3: NN_ONE(1, true); break;  // one block per wave always shares its row
        case 4: NN_ONE(2, false); break;
        case 5: NN_ONE(2, true); break;
        case 8: NN_ONE(4, false); break;
        case 9: NN_ONE(4, true); break;
        case 17:
          if constexpr (MAXNB >= 8) NN_ONE(8, true);
          else if (inf && tid == 0) *inf = nn_info_dev{0, NN_ERR_UNSUPPORTED, NAN};
          break;
        default:
          if constexpr (MAXNB >= 8) NN_ONE(8, false);
          else if (inf && tid == 0) *inf = nn_info_dev{0, NN_ERR_UNSUPPORTED, NAN};
          break;
      }
#undef NN_ONE
    } else if (!TOL && item < n_large + n_quad / 2) {
      if constexpr (!TOL) {
        // a pair of equal-size matrices, four waves each (blocks per wave 1 or 2)
        const int half = wave / kQuadWaves;
        const int b =
            __builtin_amdgcn_readfirstlane(perm[n_large + 2 * (item - n_large) + half]);
        const Group g{wave % kQuadWaves, kQuadWaves, lane, tid % (kQuadWaves * 64), half, true};
        const int64_t off = a.offsets[b] * cm, xoff = xoffsets[b] * cm;
        const int K = __builtin_amdgcn_readfirstlane(a.sizes[b]);
        const int base = half * lds_nbufs(a.depth) * quad_stride;
        nn_info_dev* inf = a.info ? a.info + b : nullptr;
        const int nbw = blocks_per_wave(K, CPLX, kQuadWaves);
        const bool sh = shared_rows(K, CPLX, nbw);
#define NN_ONE(NB, SH)                                                                       \
  invert_one<CPLX, NB, SH, TOL>(A + off, X + xoff, K, a.depth, a.x0, a.iters, a.tol, a.max_iter, \
                                base, quad_stride, g, inf)
        if (nbw == 1) NN_ONE(1, true);
        else if (sh) NN_ONE(2, true);
        else NN_ONE(2, false);
#undef NN_ONE
      }
    } else {
      const int idx = n_large + n_quad + kWaves * (item - n_large - n_quad / 2) + wave;
      if (idx < n_large + n_quad + n_small) {
        const int b = __builtin_amdgcn_readfirstlane(perm[idx]);
        const Group g{0, 1, lane, lane, wave, false};
        const int64_t off = a.offsets[b] * cm, xoff = xoffsets[b] * cm;
        const int K = __builtin_amdgcn_readfirstlane(a.sizes[b]);
        const double tol = a.tols ? a.tols[b] : a.tol;
        const int mit = a.maxits ? a.maxits[b] : a.max_iter;
        const int base = wave * lds_nbufs(a.depth) * wave_stride;
        nn_info_dev* inf = a.info ? a.info + b : nullptr;
        const int nbw = blocks_per_wave(K, CPLX, 1);
        const bool sh = shared_rows(K, CPLX, nbw);
#define NN_ONE(NB, SH)                                                                     \
  invert_one<CPLX, NB, SH, TOL>(A + off, X + xoff, K, a.depth, a.x0, a.iters, tol, mit, base, \
                                wave_stride, g, inf)
        switch (nbw * 2 + (sh ? 1 : 0)) {
          case 2:
          case 3: NN_ONE(1, true); break;  // one block per wave always shares its row
          case 4: NN_ONE(2, false); break;
          case 5: NN_ONE(2, true); break;
          case 8: NN_ONE(4, false); break;
          case 9: NN_ONE(4, true); break;
          case 17:
            if constexpr (MAXNB >= 8) NN_ONE(8, true);
            else if (inf && lane == 0) *inf = nn_info_dev{0, NN_ERR_UNSUPPORTED, NAN};
            break;
          default:
            if constexpr (MAXNB >= 8) NN_ONE(8, false);
            else if (inf && lane == 0) *inf = nn_info_dev{0, NN_ERR_UNSUPPORTED, NAN};
            break;
        }
#undef NN_ONE
      }
    }
    __syncthreads();
  }
}

size_t lds_bytes(bool cplx, int max_n, int wave_max_k, int depth) {
  const size_t nb = (size_t)lds_nbufs(depth);
  const size_t big = nb * (size_t)lds_buf(max_n, cplx);
  const int wk = wave_max_k > 0 ? wave_max_k : 1;
  const size_t small = kWaves * nb * (size_t)lds_buf(wk, cplx);  // one wave matrix per wave
  // a pair of fixed-nest matrices (counted whether or not the launch has pairs)
  const int qk = max_n < kQuadMaxK ? max_n : kQuadMaxK;
  const size_t quad = qk > wave_max_k ? 2 * nb * (size_t)lds_buf(qk, cplx) : 0;
  size_t m = big > small ? big : small;
  return sizeof(float) * (m > quad ? m : quad);
}

}  // namespace

size_t batched_ws_bytes(int32_t batch) { return 256 + ((size_t)batch * 4 + 255) / 256 * 256; }

hipError_t launch_batched(const BatchedArgs& args, hipStream_t s) {
  BatchedArgs a = args;
  BatchHdr* hdr = static_cast<BatchHdr*>(a.ws);
  int32_t* perm = reinterpret_cast<int32_t*>(static_cast<char*>(a.ws) + 256);
  const bool cplx = a.dt == NN_C64;
  if (a.wave_max_k > a.max_n) a.wave_max_k = a.max_n;
  // pairs only in the fixed-nest mode: there every matrix meets the same
  // barriers; in the tolerance mode each stops on its own
  const int qk = a.max_n < kQuadMaxK ? a.max_n : kQuadMaxK;
  a.quad_max_k = a.iters > 0 && qk > a.wave_max_k ? qk : a.wave_max_k;
  hipLaunchKernelGGL(batched_plan, dim3(1), dim3(1024), 0, s, a.sizes, a.batch, a.max_n,
                     a.wave_max_k, a.quad_max_k, hdr, perm, a.info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = lds_bytes(cplx, a.max_n, a.wave_max_k, a.depth);
  const bool nb8 = batched_max_nb(cplx, a.max_n, a.wave_max_k) > 4;
  const dim3 grid(a.grid), block(kThreads);
#define NN_LAUNCH(C, T)                                                                 \
  do {                                                                                  \
    if (nb8)                                                                            \
      hipLaunchKernelGGL((batched_nn<C, T, 8>), grid, block, lds, s, a, perm, hdr);      \
    else                                                                                \
      hipLaunchKernelGGL((batched_nn<C, T, 4>), grid, block, lds, s, a, perm, hdr);      \
  } while (0)
  if (cplx) {
    if (a.iters > 0) NN_LAUNCH(true, false);
    else NN_LAUNCH(true, true);
  } else {
    if (a.iters > 0) NN_LAUNCH(false, false);
    else NN_LAUNCH(false, true);
  }
#undef NN_LAUNCH
  return hipGetLastError();
}

int batched_max_nb(bool cplx, int max_n, int wave_max_k) {
  int m = 1;
  for (int K = 1; K <= max_n && K <= kMaxN; ++K) {
    const int nb = blocks_per_wave(K, cplx, K <= wave_max_k ? 1 : kWaves);
    m = nb > m ? nb : m;
  }
  return m;
}

size_t batched_static_lds() {
  // The persistent kernels' own LDS (the reduction rows and the work item),
  // as the compiler laid it out: 8720 bytes on gfx950 for every instantiation.
  static size_t cached = 0;
  if (!cached) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&batched_nn<true, false, 4>)) ==
            hipSuccess &&
        fa.sharedSizeBytes > 0)
      cached = fa.sharedSizeBytes;
    else
      cached = sizeof(double) * kWaves * (8 + 2 * kMaxN) + 16;
  }
  return cached;
}

int batched_fit_wave_max_k(nn_dtype dt, int max_n, int wave_max_k, int depth) {
  const bool cplx = dt == NN_C64;
  int wk = wave_max_k < max_n ? wave_max_k : max_n;
  const size_t cap = kBatchedLdsCu - batched_static_lds();
  const size_t lim = cap < kBatchedDynLds ? cap : kBatchedDynLds;
  // the one-wave sizes the kernel is tuned for, largest first
  while (wk > 0 && lds_bytes(cplx, max_n, wk, depth) > lim) wk = wk > 16 ? 16 : wk > 8 ? 8 : 0;
  return wk;
}

hipError_t batched_allow_lds() {
  const int lim = (int)kBatchedDynLds;  // dynamic part; the static part is batched_static_lds()
  const void* kernels[8] = {reinterpret_cast<const void*>(&batched_nn<true, false, 4>),
                            reinterpret_cast<const void*>(&batched_nn<true, true, 4>),
                            reinterpret_cast<const void*>(&batched_nn<false, false, 4>),
                            reinterpret_cast<const void*>(&batched_nn<false, true, 4>),
                            reinterpret_cast<const void*>(&batched_nn<true, false, 8>),
                            reinterpret_cast<const void*>(&batched_nn<true, true, 8>),
                            reinterpret_cast<const void*>(&batched_nn<false, false, 8>),
                            reinterpret_cast<const void*>(&batched_nn<false, true, 8>)};
  for (const void* k : kernels) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t batched_lds_bytes(nn_dtype dt, int max_n, int wave_max_k, int depth) {
  if (wave_max_k > max_n) wave_max_k = max_n;
  return lds_bytes(dt == NN_C64, max_n, wave_max_k, depth);
}

}  // namespace nn
