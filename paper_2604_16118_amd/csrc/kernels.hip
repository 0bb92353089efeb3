// HIP kernels for gfx950: grouped FP64 MFMA GEMM, batched Jacobi eigensolver,
// MPO W-step, block copies/scalings and a wavefront-shuffle reduction.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <stdexcept>
#include <string>

#include <type_traits>
#include "kernels.hpp"

#include <hip/hip_ext.h>

namespace pv {

typedef double d4 __attribute__((ext_vector_type(4)));

// Pointers read from descriptors are generic to the compiler, which then emits FLAT memory
// instructions; those count against the LDS wait counter as well, so every wait for an LDS
// read would also wait for outstanding global loads and stores.  Kernels therefore cast
// descriptor pointers into the global address space.
#define PV_GLOBAL __attribute__((address_space(1)))
typedef PV_GLOBAL double gdouble;
typedef PV_GLOBAL const double gcdouble;
template <class T> __device__ inline PV_GLOBAL T* gbl(T* p) { return (PV_GLOBAL T*)p; }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

#define PV_LAUNCH_CHECK()                                                          \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("kernel launch: ") + \
                                                   hipGetErrorString(e_));         \
  } while (0)

// ---------------------------------------------------------------------------
// Grouped GEMM.  One workgroup (4 waves, 2 x 2) computes a BM x BN tile of one problem;
// each wave owns a (BM/2) x (BN/2) quadrant as (BM/32) x (BN/32) tiles of
// v_mfma_f64_16x16x4f64 (or v_mfma_f32_16x16x4f32 in the float32 variant).  Operand
// layout of both (wave64): lane l supplies A[l%16][l/16] and B[l/16][l%16]; the 16x16
// result lives in 4 values per lane, element r of lane l being D[4r + l/16][l%16] for
// float64 and D[4(l/16) + r][l%16] for float32 (both measured with single-instruction
// probes on gfx950).  The tile is 64 x 64 (BM x BN): measured on the L=48 workload, 128 x 64,
// 64 x 128 and larger tiles lose more to the lower occupancy than they save in re-reads.
// ---------------------------------------------------------------------------
// XCD-aware order: workgroup b runs on XCD b % 8.  Tiles are dealt to the XCDs in groups of
// kGemmGroup consecutive ones (same row block of A, consecutive column blocks), so a group
// shares one L2 while every XCD still gets an even mix of the problems; the ragged end keeps
// the plain order.
__device__ inline int gemm_tile_of_block(int ntiles) {
  const int b = blockIdx.x, span = 8 * kGemmGroup;
  int tile = b;
  if (b < ntiles / span * span) {
    const int base = b - b % span, r = b - base;
    tile = base + (r & 7) * kGemmGroup + (r >> 3);
  }
  return tile;
}

template <int PREC, int BM, int BN>
__device__ __forceinline__ void gemm_tile(const GemmDesc& g, int tile) {
  // PREC 0: float64 operands on v_mfma_f64_16x16x4f64; PREC 1: operands rounded to float32
  // on v_mfma_f32_16x16x4f32 with float32 accumulation (C stays float64 in memory);
  // PREC 2: the float64 kernel again, a separate instance for the trailing updates of the
  // tridiagonal reduction so that profiles tell the two uses apart
  constexpr bool F64 = PREC != 1;
  typedef typename std::conditional<F64, double, float>::type T;
  constexpr int BK = kGemmBK;
  constexpr int KS = BK / 4;                             // MFMA k-steps per K-tile
  constexpr int TM = BM / 32, TN = BN / 32;              // MFMA tiles per wave
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;  // elements per thread per K-tile
  // double-buffered K-tiles: the global loads of tile t+1 are held in registers while the
  // MFMAs of tile t run, then written to the other LDS buffer (one barrier per K-tile)
  __shared__ T As[2][BK][BM + 1];
  __shared__ T Bs[2][BK][BN + 1];
  gcdouble* gA = gbl(g.A);
  gcdouble* gB = gbl(g.B);
  gdouble* gC = gbl(g.C);
  const int t = tile - g.tile0;
  const int row0 = (g.colmajor ? t % g.tiles_m : t / g.tiles_n) * BM;
  const int col0 = (g.colmajor ? t / g.tiles_m : t % g.tiles_n) * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  // the wavefront index is uniform: taken from the first lane it lives in a scalar
  // register, so the sub-tile conditions below are scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  // per-thread element coordinates inside a K-tile (fastest index along contiguous memory)
  int ai[LA], ak[LA], bj[LB], bk[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int e = tid + 256 * r;
    if (!g.ta) { ai[r] = e % BM; ak[r] = e / BM; } else { ak[r] = e % BK; ai[r] = e / BK; }
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int e = tid + 256 * r;
    if (!g.tb) { bk[r] = e % BK; bj[r] = e / BK; } else { bj[r] = e % BN; bk[r] = e / BN; }
  }
  // out-of-range elements load from a clamped (valid) address and are replaced by zero
  // when they are written to LDS, so the loads are straight-line code whose results are
  // first needed at the end of the K-tile
  // the row (of A) and column (of B) part of each thread's addresses is fixed for the tile
  const int64_t sAi = g.ta ? g.lda : 1, sAk = g.ta ? 1 : g.lda;
  const int64_t sBj = g.tb ? 1 : g.ldb, sBk = g.tb ? g.ldb : 1;
  gcdouble* pa[LA];
  gcdouble* pb[LB];
  bool rowa[LA], colb[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int gi = row0 + ai[r];
    rowa[r] = gi < g.M;
    const int ci = min(gi, g.M - 1);
    pa[r] = g.m1 > 0 ? gA + (ci % g.m1) + (int64_t)(ci / g.m1) * g.a_outer : gA + ci * sAi;
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int gj = col0 + bj[r];
    colb[r] = gj < g.N;
    pb[r] = gB + min(gj, g.N - 1) * sBj;
  }
  double ra[LA], rb[LB];
  bool oka[LA], okb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gk = k0 + ak[r];
      oka[r] = rowa[r] && gk < g.kend;
      ra[r] = pa[r][min(gk, g.kend - 1) * sAk];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gk = k0 + bk[r];
      okb[r] = colb[r] && gk < g.kend;
      rb[r] = pb[r][min(gk, g.kend - 1) * sBk];
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) As[buf][ak[r]][ai[r]] = oka[r] ? T(ra[r]) : T(0);
#pragma unroll
    for (int r = 0; r < LB; ++r) Bs[buf][bk[r]][bj[r]] = okb[r] ? T(rb[r]) : T(0);
  };
  typedef T T4 __attribute__((ext_vector_type(4)));
  T4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = T4{0, 0, 0, 0};
  // 16 x 16 sub-tiles that lie wholly outside C (edge tiles of a problem) are skipped;
  // interior tiles run a loop without any condition around the MFMAs
  bool rv[TM], cv[TN];
  bool full = true;
#pragma unroll
  for (int a = 0; a < TM; ++a) { rv[a] = row0 + wr * (BM / 2) + a * 16 < g.M; full = full && rv[a]; }
#pragma unroll
  for (int b = 0; b < TN; ++b) { cv[b] = col0 + wc * (BN / 2) + b * 16 < g.N; full = full && cv[b]; }
  auto kloop = [&](auto all_valid) {
    int buf = 0;
    for (int k0 = g.kbeg; k0 < g.kend; k0 += BK) {
      const bool more = k0 + BK < g.kend;
      if (more) load(k0 + BK);
      // fragments of the next k-step are read from LDS before the MFMAs of the current one
      T af[2][TM], bf[2][TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) af[0][a] = As[buf][lk][wr * (BM / 2) + a * 16 + li];
#pragma unroll
      for (int b = 0; b < TN; ++b) bf[0][b] = Bs[buf][lk][wc * (BN / 2) + b * 16 + li];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < KS) {
#pragma unroll
          for (int a = 0; a < TM; ++a) af[cur ^ 1][a] = As[buf][4 * (ks + 1) + lk][wr * (BM / 2) + a * 16 + li];
#pragma unroll
          for (int b = 0; b < TN; ++b) bf[cur ^ 1][b] = Bs[buf][4 * (ks + 1) + lk][wc * (BN / 2) + b * 16 + li];
        }
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b) {
            if constexpr (!decltype(all_valid)::value) {
              if (!(rv[a] && cv[b])) continue;
            }
            if constexpr (F64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[cur][a], bf[cur][b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[cur][a], bf[cur][b], acc[a][b], 0, 0, 0);
          }
      }
      if (more) stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  };
  if (g.kbeg < g.kend) {
    load(g.kbeg);
    stage(0);
  }
  __syncthreads();
  if (full) kloop(std::true_type{});
  else kloop(std::false_type{});
  // result element r of lane l: row 4r + l/16 (float64 instruction), row 4 (l/16) + r
  // (float32 instruction), column l % 16 (measured on gfx950).  With beta != 0 all loads of C
  // are issued before any is used, so their latencies overlap.
  auto row_of = [&](int mi, int r) { return row0 + wr * (BM / 2) + mi * 16 + (F64 ? 4 * r + lk : 4 * lk + r); };
  auto col_of = [&](int nj) { return col0 + wc * (BN / 2) + nj * 16 + li; };
  // offset of row i of C (two-level rows when m1 > 0)
  int64_t crow[TM][4];
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ic = min(row_of(mi, r), g.M - 1);
      crow[mi][r] = g.m1 > 0 ? (ic % g.m1) + (int64_t)(ic / g.m1) * g.c_outer : (int64_t)ic;
    }
  double cold[TM][TN][4];
  if (g.beta != 0.0) {
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int nj = 0; nj < TN; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int jc = min(col_of(nj), g.N - 1);
          cold[mi][nj][r] = gC[crow[mi][r] + (int64_t)jc * g.ldc];
        }
  }
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int nj = 0; nj < TN; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row_of(mi, r), j = col_of(nj);
        if (i < g.M && j < g.N) {
          double v = g.alpha * double(acc[mi][nj][r]);
          if (g.beta != 0.0) v += g.beta * cold[mi][nj][r];
          gC[crow[mi][r] + (int64_t)j * g.ldc] = v;
        }
      }
}

// bfloat16 bits of a double, rounded to nearest even through float (the standard bit
// formula on the float: add 0x7fff plus the lowest kept bit, keep the upper half)
__device__ inline unsigned short bf16_bits(double x) {
  const float f = float(x);
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// PREC 3: operands rounded to bfloat16 on v_mfma_f32_16x16x16_bf16 (one instruction per
// 16 x 16 sub-tile and K-tile of 16), float32 accumulation, C float64 in memory.  The LDS
// tiles hold each row (of A) or column (of B) with its 16 k values contiguous, so that a
// lane reads its four consecutive k values of a sub-tile with one 8-byte load.  The
// instruction pairs the A and B values of the same (lane group, element), so the sum over
// k does not depend on which k the hardware assigns to them; rows of A and columns of B
// are lane % 16 and the result layout is that of the float32 instruction.
template <int BM, int BN>
__device__ __forceinline__ void gemm_tile_bf16(const GemmDesc& g, int tile) {
  constexpr int BK = kGemmBK;
  static_assert(BK == 16, "one bf16 MFMA per K-tile");
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  constexpr int KP = BK + 4;  // row pitch in bf16 elements (8-byte aligned rows)
  __shared__ unsigned short As[2][BM][KP];
  __shared__ unsigned short Bs[2][BN][KP];
  gcdouble* gA = gbl(g.A);
  gcdouble* gB = gbl(g.B);
  gdouble* gC = gbl(g.C);
  const int t = tile - g.tile0;
  const int row0 = (g.colmajor ? t % g.tiles_m : t / g.tiles_n) * BM;
  const int col0 = (g.colmajor ? t / g.tiles_m : t % g.tiles_n) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  int ai[LA], ak[LA], bj[LB], bk[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int e = tid + 256 * r;
    if (!g.ta) { ai[r] = e % BM; ak[r] = e / BM; } else { ak[r] = e % BK; ai[r] = e / BK; }
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int e = tid + 256 * r;
    if (!g.tb) { bk[r] = e % BK; bj[r] = e / BK; } else { bj[r] = e % BN; bk[r] = e / BN; }
  }
  double ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gi = row0 + ai[r], gk = k0 + ak[r];
      ra[r] = (gi < g.M && gk < g.kend) ? (g.ta ? gA[gk + (int64_t)gi * g.lda] : gA[gi + (int64_t)gk * g.lda]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gj = col0 + bj[r], gk = k0 + bk[r];
      rb[r] = (gj < g.N && gk < g.kend) ? (g.tb ? gB[gj + (int64_t)gk * g.ldb] : gB[gk + (int64_t)gj * g.ldb]) : 0.0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) As[buf][ai[r]][ak[r]] = bf16_bits(ra[r]);
#pragma unroll
    for (int r = 0; r < LB; ++r) Bs[buf][bj[r]][bk[r]] = bf16_bits(rb[r]);
  };
  typedef float F4 __attribute__((ext_vector_type(4)));
  typedef short S4 __attribute__((ext_vector_type(4)));
  F4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = F4{0, 0, 0, 0};
  bool rv[TM], cv[TN];
#pragma unroll
  for (int a = 0; a < TM; ++a) rv[a] = row0 + wr * (BM / 2) + a * 16 < g.M;
#pragma unroll
  for (int b = 0; b < TN; ++b) cv[b] = col0 + wc * (BN / 2) + b * 16 < g.N;
  int buf = 0;
  if (g.kbeg < g.kend) {
    load(g.kbeg);
    stage(0);
  }
  __syncthreads();
  for (int k0 = g.kbeg; k0 < g.kend; k0 += BK) {
    const bool more = k0 + BK < g.kend;
    if (more) load(k0 + BK);
    S4 af[TM], bf[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
      af[a] = *reinterpret_cast<const S4*>(&As[buf][wr * (BM / 2) + a * 16 + li][4 * lk]);
#pragma unroll
    for (int b = 0; b < TN; ++b)
      bf[b] = *reinterpret_cast<const S4*>(&Bs[buf][wc * (BN / 2) + b * 16 + li][4 * lk]);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        if (!(rv[a] && cv[b])) continue;
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  auto row_of = [&](int mi, int r) { return row0 + wr * (BM / 2) + mi * 16 + 4 * lk + r; };
  auto col_of = [&](int nj) { return col0 + wc * (BN / 2) + nj * 16 + li; };
  double cold[TM][TN][4];
  if (g.beta != 0.0) {
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int nj = 0; nj < TN; ++nj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = row_of(mi, r), j = col_of(nj);
          const int ic = min(i, g.M - 1), jc = min(j, g.N - 1);
          cold[mi][nj][r] = gC[ic + (int64_t)jc * g.ldc];
        }
  }
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int nj = 0; nj < TN; ++nj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = row_of(mi, r), j = col_of(nj);
        if (i < g.M && j < g.N) {
          double v = g.alpha * double(acc[mi][nj][r]);
          if (g.beta != 0.0) v += g.beta * cold[mi][nj][r];
          gC[i + (int64_t)j * g.ldc] = v;
        }
      }
}

template <int PREC, int BM, int BN>
__device__ __forceinline__ void gemm_any(const GemmDesc& g, int tile) {
  if constexpr (PREC == 3) gemm_tile_bf16<BM, BN>(g, tile);
  else gemm_tile<PREC, BM, BN>(g, tile);
}

// tmap[tile] is the problem of each tile: one load instead of a search over the
// descriptors (batches reach thousands of problems of a few tiles each, where a chain of
// dependent descriptor loads costs as much as the tile's own K loop)
template <int PREC, int BM, int BN>
__global__ __launch_bounds__(256, 4) void gemm_kernel(const GemmDesc* __restrict__ descs, const int* __restrict__ tmap,
                                                   int ntiles) {
  const int tile = gemm_tile_of_block(ntiles);
  const GemmDesc g = descs[tmap[tile]];
  gemm_any<PREC, BM, BN>(g, tile);
}

// The same with the descriptors in the kernel arguments (at most kGemmPack problems): no
// upload has to precede the launch.
template <int PREC, int BM, int BN>
__global__ __launch_bounds__(256, 4) void gemm_packed_kernel(const GemmPack pack, int nprob, int ntiles) {
  const int tile = gemm_tile_of_block(ntiles);
  int lo = 0;
  for (int p = 1; p < nprob; ++p)
    if (pack.d[p].tile0 <= tile) lo = p;
  const GemmDesc g = pack.d[lo];
  gemm_any<PREC, BM, BN>(g, tile);
}

// The events, when given, take the launch's own start and stop times (an extended launch:
// no marker packets around it, so they time the kernel's execution alone).
void launch_gemm_packed(const GemmPack& pack, int nprob, int total_tiles, int prec, hipStream_t s, bool small,
                        hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (total_tiles <= 0) return;
  if (nprob < 1 || nprob > kGemmPack) throw std::runtime_error("gemm: a packed launch takes 1 to kGemmPack problems");
  if (small && prec != 0 && prec != 2) throw std::runtime_error("gemm: small tiles are float64 only");
  const dim3 g(total_tiles), b(256);
  auto go = [&](auto kernel) {
    hipExtLaunchKernelGGL(kernel, g, b, 0, s, ev_start, ev_stop, 0, pack, nprob, total_tiles);
  };
  if (small && prec == 0)
    go(gemm_packed_kernel<0, kGemmSmall, kGemmSmall>);
  else if (small)
    go(gemm_packed_kernel<2, kGemmSmall, kGemmSmall>);
  else if (prec == 0)
    go(gemm_packed_kernel<0, kGemmBM, kGemmBN>);
  else if (prec == 1)
    go(gemm_packed_kernel<1, kGemmBM, kGemmBN>);
  else if (prec == 3)
    go(gemm_packed_kernel<3, kGemmBM, kGemmBN>);
  else
    go(gemm_packed_kernel<2, kGemmBM, kGemmBN>);
  PV_LAUNCH_CHECK();
}

void launch_gemm(const GemmDesc* d_desc, const int* d_tmap, int total_tiles, int prec, hipStream_t s, bool small,
                 hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (total_tiles <= 0) return;
  if (small && prec != 0 && prec != 2) throw std::runtime_error("gemm: small tiles are float64 only");
  const dim3 g(total_tiles), b(256);
  auto go = [&](auto kernel) {
    hipExtLaunchKernelGGL(kernel, g, b, 0, s, ev_start, ev_stop, 0, d_desc, d_tmap, total_tiles);
  };
  if (small && prec == 0)
    go(gemm_kernel<0, kGemmSmall, kGemmSmall>);
  else if (small)
    go(gemm_kernel<2, kGemmSmall, kGemmSmall>);
  else if (prec == 0)
    go(gemm_kernel<0, kGemmBM, kGemmBN>);
  else if (prec == 1)
    go(gemm_kernel<1, kGemmBM, kGemmBN>);
  else if (prec == 3)
    go(gemm_kernel<3, kGemmBM, kGemmBN>);
  else
    go(gemm_kernel<2, kGemmBM, kGemmBN>);
  PV_LAUNCH_CHECK();
}

__global__ void reduce_kernel(const ReduceDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const ReduceDesc r = d[lo];
  const int64_t x = e - r.elem0;
  const int i = int(x % r.M), j = int(x / r.M);
  const int64_t mn = (int64_t)r.M * r.N;
  double acc = 0.0;
  gcdouble* P = gbl(r.P);
  for (int s = 0; s < r.S; ++s) acc += P[s * mn + x];
  gdouble* c = gbl(r.C) + i + (int64_t)j * r.ldc;
  double v = r.alpha * acc;
  if (r.beta != 0.0) v += r.beta * *c;
  *c = v;
}

void launch_reduce(const ReduceDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Cyclic two-sided Jacobi eigensolver, one workgroup per matrix.
// Parallel ordering: the circle method pairs the n2 (= n rounded up to even) indices
// into n2/2 disjoint pairs per step, n2-1 steps per sweep meeting every pair once.
// All rotations of a step are applied at once as 2x2 block updates
// B_ij <- J_i^T B_ij J_j over the block rows/columns of the pairs.  The working
// matrix is the packed upper triangle; depending on the size it lives in LDS together
// with V (MODE 2), in LDS with V in global memory (MODE 1), or both in global memory
// (MODE 0).  A rotation is applied when |a_pq| > 1e-14 sqrt(|a_pp a_qq|) and
// |a_pq| > abs_tol max_i |a_ii|.  On a general matrix the updates leave rounding noise
// of order eps max|a_ii| in the small-eigenvalue block, which the relative test alone
// keeps rotating; an absolute floor above that noise (abs_tol = 1e-15) ends the sweeps.
// On nearly diagonal input (the second pass of a two-pass factorisation) the noise is
// local and abs_tol = 0 keeps small eigenvalues relatively accurate.  Sweeps stop when a
// sweep applies no rotation.
// ---------------------------------------------------------------------------
constexpr int kEigMaxPairs = kEigMax / 2;
constexpr double kJacobiTol = 1e-14;

__device__ inline int pidx(int r, int c) {  // packed upper, r <= c (n <= 1024: fits int32)
  return (c * (c + 1) >> 1) + r;
}
__device__ inline int sidx(int r, int c) { return r <= c ? pidx(r, c) : pidx(c, r); }

// Dynamic LDS of one problem in each mode (bytes).
__host__ __device__ inline size_t eig_lds_bytes(int n, int mode) {
  const int P = (n + (n & 1)) / 2;
  size_t b = size_t(P) * (2 * sizeof(double) + 2 * sizeof(int));
  if (mode >= 1) b += size_t(n) * (n + 1) / 2 * sizeof(double);
  if (mode == 2) b += size_t(n) * n * sizeof(double);
  return b;
}

constexpr int kEigBlocksPerThread = 8;  // (P(P+1)/2) / threads <= 8 for n <= 1024 at 1024 threads
                                        // is not guaranteed; larger counts fall back to a loop

template <int MODE>
__global__ __launch_bounds__(1024) void jacobi_eig_kernel(const EigDesc* __restrict__ descs, int maxsweep) {
  extern __shared__ double smem[];
  __shared__ int rotated;
  __shared__ double dmax;
  const EigDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int n2 = n + (n & 1), P = n2 / 2;
  double* lds = smem;
  double* Ap;
  double* Vw;
  if (MODE == 0) { Vw = d.work; Ap = d.work + (int64_t)n * n; }
  else if (MODE == 1) { Vw = d.work; Ap = lds; lds += n * (n + 1) / 2; }
  else { Ap = lds; lds += n * (n + 1) / 2; Vw = lds; lds += n * n; }
  double* rc = lds;
  double* rs = rc + P;
  int* rp = reinterpret_cast<int*>(rs + P);
  int* rq = rp + P;
  for (int c = 0; c < n; ++c)
    for (int r = tid; r <= c; r += bs) Ap[pidx(r, c)] = d.A[r + (int64_t)c * d.lda];
  for (int e = tid; e < n * n; e += bs) {
    const int col = e / n;
    Vw[e] = (e - col * n == col) ? 1.0 : 0.0;
  }
  // this thread's 2x2 blocks (i <= j) of the pair-indexed matrix, decoded once
  const int nb = P * (P + 1) / 2;
  int myblk[kEigBlocksPerThread];
  int nmine = 0;
  for (int e = tid; e < nb && nmine < kEigBlocksPerThread; e += bs) {
    int j = int((sqrtf(8.0f * float(e) + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    while (j * (j + 1) / 2 > e) --j;
    myblk[nmine++] = ((e - j * (j + 1) / 2) << 16) | j;
  }
  const int extra_start = tid + kEigBlocksPerThread * bs;  // blocks beyond the cached ones
  __syncthreads();
  int sweeps = 0;
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    if (tid == 0) {
      rotated = 0;
      double m = 0.0;
      for (int i = 0; i < n; ++i) m = fmax(m, fabs(Ap[pidx(i, i)]));
      dmax = m;
    }
    __syncthreads();
    ++sweeps;
    const double abs_floor = fmax(d.abs_tol * dmax, 1e-300);
    for (int step = 0; step < n2 - 1; ++step) {
      for (int k = tid; k < P; k += bs) {
        int a, b;
        if (k == 0) { a = n2 - 1; b = step; }
        else {
          a = step + k; if (a >= n2 - 1) a -= n2 - 1;
          b = step - k; if (b < 0) b += n2 - 1;
        }
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = Ap[pidx(p, p)], aqq = Ap[pidx(q, q)], apq = Ap[pidx(p, q)];
          if (fabs(apq) > kJacobiTol * sqrt(fabs(app * aqq)) && fabs(apq) > abs_floor) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        rp[k] = p; rq[k] = q; rc[k] = c; rs[k] = s;
      }
      __syncthreads();
      auto update = [&](int i, int j) {
        const double si = rs[i], sj = rs[j];
        if (si == 0.0 && sj == 0.0) return;
        const double ci = rc[i], cj = rc[j];
        const int pi = rp[i], qi = rq[i], pj = rp[j], qj = rq[j];
        if (i == j) {
          if (qi >= n) return;
          const double app = Ap[pidx(pi, pi)], aqq = Ap[pidx(qi, qi)], apq = Ap[pidx(pi, qi)];
          Ap[pidx(pi, pi)] = ci * ci * app - 2.0 * ci * si * apq + si * si * aqq;
          Ap[pidx(qi, qi)] = si * si * app + 2.0 * ci * si * apq + ci * ci * aqq;
          Ap[pidx(pi, qi)] = 0.0;
        } else {
          const bool vqi = qi < n, vqj = qj < n;
          const double b00 = Ap[sidx(pi, pj)];
          const double b01 = vqj ? Ap[sidx(pi, qj)] : 0.0;
          const double b10 = vqi ? Ap[sidx(qi, pj)] : 0.0;
          const double b11 = (vqi && vqj) ? Ap[sidx(qi, qj)] : 0.0;
          const double t00 = ci * b00 - si * b10, t01 = ci * b01 - si * b11;
          const double t10 = si * b00 + ci * b10, t11 = si * b01 + ci * b11;
          Ap[sidx(pi, pj)] = t00 * cj - t01 * sj;
          if (vqj) Ap[sidx(pi, qj)] = t00 * sj + t01 * cj;
          if (vqi) Ap[sidx(qi, pj)] = t10 * cj - t11 * sj;
          if (vqi && vqj) Ap[sidx(qi, qj)] = t10 * sj + t11 * cj;
        }
      };
      for (int m = 0; m < nmine; ++m) update(myblk[m] >> 16, myblk[m] & 0xffff);
      for (int e = extra_start; e < nb; e += bs) {
        int j = int((sqrtf(8.0f * float(e) + 1.0f) - 1.0f) * 0.5f);
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        while (j * (j + 1) / 2 > e) --j;
        update(e - j * (j + 1) / 2, j);
      }
      for (int e = tid; e < P * n; e += bs) {
        const int k = e / n, r = e - k * n;
        const double s = rs[k];
        if (s == 0.0) continue;
        const double c = rc[k];
        double* vp = Vw + rp[k] * n + r;
        double* vq = Vw + rq[k] * n + r;
        const double x = *vp, y = *vq;
        *vp = c * x - s * y;
        *vq = s * x + c * y;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // eigenvalues, sorted descending (ties: lower index first), and matching vectors
  for (int i = tid; i < n; i += bs) {
    const double wi = Ap[pidx(i, i)];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = Ap[pidx(j, j)];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    d.w[rank] = wi;
    for (int r = 0; r < n; ++r) d.V[r + (int64_t)rank * n] = Vw[r + i * n];
  }
  if (tid == 0 && d.sweeps) *d.sweeps = sweeps;
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver by Householder tridiagonalisation, multisection and inverse
// iteration (used for the Gram eigenproblems of the scaled path, where Jacobi's O(n^3)
// traffic per sweep is too slow):
//  1. A = Q T Q^T with Householder reflectors H_k = I - beta_k v_k v_k^T acting on rows
//     and columns k+1..n-1 (the trailing block is updated by the symmetric rank-2 form
//     A <- A - v q^T - q v^T, q = p - (beta/2)(v^T p) v, p = beta A v), blocked in panels
//     of kTriPanel columns whose trailing updates are GEMMs;
//  2. every eigenvalue of T by multisection on the Sturm count (a group of lanes per
//     eigenvalue);
//  3. eigenvectors of T by inverse iteration with a partially pivoted tridiagonal LU: two
//     solves for an isolated eigenvalue, three for the members of a cluster (gap <= 1e-7
//     ||T||), which the workgroup orthogonalises against each other by classical
//     Gram-Schmidt applied twice; eigenvalues <= vec_cut * max |lambda| get a zero vector
//     (the callers drop them);
//  4. back-transformation V = H_0 H_1 ... H_{n-3} Z, in which every wavefront carries two
//     columns of Z in registers through all reflectors (no workgroup barriers, n/8
//     workgroups per matrix; four columns per wavefront, with half the waves, measured
//     slower).
// Each phase is its own launch with its own register budget.  Output as the Jacobi kernel: eigenvalues descending, eigenvectors
// in the columns of V.
// ---------------------------------------------------------------------------
constexpr int kTriThreads = 1024;
constexpr int kValuesThreads = 256;  // threads per workgroup of the bisection
// Multisection: kSectLanes lanes of a wavefront share one eigenvalue and each evaluates the
// Sturm count at kSectPoints points per round (interleaved, so their latencies overlap); a
// round cuts the bracket into kSectLanes * kSectPoints + 1 equal parts, four bits instead
// of the one bit of bisection, and so shortens each eigenvalue's chain of dependent sweeps.
constexpr int kSectLanes = 8;
constexpr int kSectPoints = 2;
constexpr int kSectQ = kSectLanes * kSectPoints;
constexpr int kValuesPositions = kValuesThreads / kSectLanes;  // eigenvalues per workgroup
// batches of at most this many eigenvalues in all take a wavefront per eigenvalue
constexpr int64_t kSectWideMax = 4096;
static_assert(64 % kSectLanes == 0, "a multisection group lies within one wavefront");
constexpr int kVectorPositions = 64;   // eigenvectors (threads) per workgroup of inverse iteration
constexpr int kBackRows = kEigMax / 64;  // rows per lane when a wavefront holds a column

__device__ inline double block_sum(double v, double* red, int tid, int bs) {
  v = wave_sum_d(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (bs + 63) / 64; ++w) t += red[w];
  return t;
}

// Number of eigenvalues of T below x (negative pivots of the LDL^T factorisation of T - x)
// at P points at once, the P recurrences interleaved so that their latencies overlap.
// Pivots smaller than tiny in magnitude are replaced by -tiny; 1/q comes from the hardware
// reciprocal refined by two Newton steps r <- r (2 - q r), which leaves a relative error of
// a few ulps (a small relative perturbation of e_i^2, as the division itself makes).
template <int P>
__device__ inline void sturm_counts(const double* d, const double* e2, int n, const double (&x)[P], double tiny,
                                    int (&cnt)[P]) {
  double q[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    q[p] = d[0] - x[p];
    if (fabs(q[p]) < tiny) q[p] = -tiny;
    cnt[p] = q[p] < 0.0;
  }
  auto step = [&](double di, double ei) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double r = __builtin_amdgcn_rcp(q[p]);
      r = r * fma(-q[p], r, 2.0);
      r = r * fma(-q[p], r, 2.0);
      q[p] = (di - x[p]) - ei * r;
      if (fabs(q[p]) < tiny) q[p] = -tiny;
      cnt[p] += q[p] < 0.0;
    }
  };
  // the LDS operands of four steps are read before the first of them is used
  int i = 1;
  for (; i + 4 <= n; i += 4) {
    const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    step(d0, f0);
    step(d1, f1);
    step(d2, f2);
    step(d3, f3);
  }
  for (; i < n; ++i) step(d[i], e2[i - 1]);
}

// Solve (T - sigma I) x = b in place for one thread: LU with partial pivoting of the
// tridiagonal matrix (the pivot rows carry one extra superdiagonal).  Every array has
// element i at [i * ld]: slots of neighbouring threads are interleaved so that a
// wavefront's accesses are contiguous.  u holds the reciprocals of the pivots.
__device__ void tri_factor(const double* d, const double* e, int n, double sigma, double tiny,
                           gdouble* u, gdouble* v, gdouble* w, gdouble* mult, gdouble* piv, int64_t ld) {
  double cd = d[0] - sigma, cs1 = n > 1 ? e[0] : 0.0, cs2 = 0.0;
  // both cases of the pivot choice by selects (one division per step, no divergence
  // between the lanes, which take different choices): no interchange, m = sub / cd (0 for
  // cd = 0); interchange, m = cd / sub
  // The pivot is den in both cases, so one reciprocal serves the multiplier and u: the
  // hardware estimate refined by two Newton steps r <- r + r (1 - den r) (a few ulps,
  // like a rounding of m and u), a shorter dependent chain than an IEEE division.
  auto step = [&](int i, double sub, double a1, double s1) {
    const bool sw = !(fabs(cd) >= fabs(sub));
    const double num = sw ? cd : sub, den = sw ? sub : cd;
    const double dz = den == 0.0 ? tiny : den;
    double r = __builtin_amdgcn_rcp(dz);
    r = fma(r, fma(-dz, r, 1.0), r);
    r = fma(r, fma(-dz, r, 1.0), r);
    const double m = (sw || cd != 0.0) ? num * r : 0.0;
    piv[i * ld] = sw ? 1.0 : 0.0;
    mult[i * ld] = m;
    const double vi = sw ? a1 : cs1, wi = sw ? s1 : cs2;
    const double ncd = sw ? cs1 - m * a1 : a1 - m * cs1;
    const double ncs = sw ? cs2 - m * s1 : s1 - m * cs2;
    cd = ncd;
    cs1 = ncs;
    cs2 = 0.0;
    u[i * ld] = r;
    v[i * ld] = vi;
    w[i * ld] = wi;
  };
  // the LDS operands of four steps are read before the first of them is used
  int i = 0;
  for (; i + 4 < n - 1; i += 4) {
    double sb[4], a[4], s[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      sb[b] = e[i + b];
      a[b] = d[i + b + 1] - sigma;
      s[b] = e[i + b + 1];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) step(i + b, sb[b], a[b], s[b]);
  }
  for (; i < n - 1; ++i) step(i, e[i], d[i + 1] - sigma, (i + 1 < n - 1) ? e[i + 1] : 0.0);
  u[(n - 1) * ld] = 1.0 / (cd == 0.0 ? tiny : cd);
  v[(n - 1) * ld] = 0.0;
  w[(n - 1) * ld] = 0.0;
}

// Solve with the factors of tri_factor for the right-hand side scale * x, in place; returns
// the squared norm of the solution.  The loads of kSolveBatch rows are issued before the
// first of them is used, so a pass waits once per batch rather than once per row; and the
// loads of the next batch are issued before the current batch's results are stored: loads
// and stores share one in-order memory counter, so a wait for loads issued after stores
// would also wait for the stores to be acknowledged.
constexpr int kSolveBatch = 8;
__device__ double tri_solve(int n, gcdouble* u, gcdouble* v, gcdouble* w, gcdouble* mult, gcdouble* piv, gdouble* x,
                            int64_t ld, double scale) {
  constexpr int B = kSolveBatch;
  // forward: apply the row operations to the right-hand side
  double cur = scale * x[0];
  auto forward = [&](int i, double nx, double m, double pv) {
    const double nxt = scale * nx;
    const bool sw = pv != 0.0;  // rows interchanged at step i
    x[i * ld] = sw ? nxt : cur;
    cur = sw ? cur - m * nxt : nxt - m * cur;
  };
  const int nbf = (n - 1) / B;  // full batches over rows 0 .. n - 2
  {
    double nx0[B], mm0[B], pp0[B], nx1[B], mm1[B], pp1[B];
    auto ld0 = [&](int i) {
#pragma unroll
      for (int b = 0; b < B; ++b) { nx0[b] = x[(i + 1 + b) * ld]; mm0[b] = mult[(i + b) * ld]; pp0[b] = piv[(i + b) * ld]; }
    };
    auto ld1 = [&](int i) {
#pragma unroll
      for (int b = 0; b < B; ++b) { nx1[b] = x[(i + 1 + b) * ld]; mm1[b] = mult[(i + b) * ld]; pp1[b] = piv[(i + b) * ld]; }
    };
    if (nbf > 0) ld0(0);
    for (int k = 0; k < nbf; k += 2) {
      const int i = k * B;
      if (k + 1 < nbf) ld1(i + B);
#pragma unroll
      for (int b = 0; b < B; ++b) forward(i + b, nx0[b], mm0[b], pp0[b]);
      if (k + 1 >= nbf) break;
      if (k + 2 < nbf) ld0(i + 2 * B);
#pragma unroll
      for (int b = 0; b < B; ++b) forward(i + B + b, nx1[b], mm1[b], pp1[b]);
    }
  }
  for (int i = nbf * B; i < n - 1; ++i) forward(i, x[(i + 1) * ld], mult[i * ld], piv[i * ld]);
  // back substitution
  double x1 = cur * u[(n - 1) * ld];
  x[(n - 1) * ld] = x1;
  double q = x1 * x1;
  if (n < 2) return q;
  double x0 = (x[(n - 2) * ld] - v[(n - 2) * ld] * x1) * u[(n - 2) * ld];
  x[(n - 2) * ld] = x0;
  q += x0 * x0;
  auto backward = [&](int r, double xr, double vr, double wr, double ur) {
    const double xi = (xr - vr * x0 - wr * x1) * ur;
    x[r * ld] = xi;
    q += xi * xi;
    x1 = x0;
    x0 = xi;
  };
  // rows n - 3 down to 0 in batches of B (row i - b of the batch starting at i)
  const int nbb = (n - 2) / B;
  {
    double xx0[B], vv0[B], ww0[B], uu0[B], xx1[B], vv1[B], ww1[B], uu1[B];
    auto lb0 = [&](int i) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int64_t o = (i - b) * ld;
        xx0[b] = x[o]; vv0[b] = v[o]; ww0[b] = w[o]; uu0[b] = u[o];
      }
    };
    auto lb1 = [&](int i) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int64_t o = (i - b) * ld;
        xx1[b] = x[o]; vv1[b] = v[o]; ww1[b] = w[o]; uu1[b] = u[o];
      }
    };
    if (nbb > 0) lb0(n - 3);
    for (int k = 0; k < nbb; k += 2) {
      const int i = n - 3 - k * B;
      if (k + 1 < nbb) lb1(i - B);
#pragma unroll
      for (int b = 0; b < B; ++b) backward(i - b, xx0[b], vv0[b], ww0[b], uu0[b]);
      if (k + 1 >= nbb) break;
      if (k + 2 < nbb) lb0(i - 2 * B);
#pragma unroll
      for (int b = 0; b < B; ++b) backward(i - B - b, xx1[b], vv1[b], ww1[b], uu1[b]);
    }
  }
  for (int i = n - 3 - nbb * B; i >= 0; --i) backward(i, x[i * ld], v[i * ld], w[i * ld], u[i * ld]);
  return q;
}

// x <- scale * x for n elements at stride ld, kSolveBatch loads at a time, each batch's
// loads issued before the previous batch's stores.
__device__ void strided_scale(int n, gdouble* x, int64_t ld, double scale) {
  constexpr int B = kSolveBatch;
  const int nb = n / B;
  double a0[B], a1[B];
  if (nb > 0)
#pragma unroll
    for (int b = 0; b < B; ++b) a0[b] = x[b * ld];
  for (int k = 0; k < nb; k += 2) {
    const int i = k * B;
    if (k + 1 < nb)
#pragma unroll
      for (int b = 0; b < B; ++b) a1[b] = x[(i + B + b) * ld];
#pragma unroll
    for (int b = 0; b < B; ++b) x[(i + b) * ld] = scale * a0[b];
    if (k + 1 >= nb) break;
    if (k + 2 < nb)
#pragma unroll
      for (int b = 0; b < B; ++b) a0[b] = x[(i + 2 * B + b) * ld];
#pragma unroll
    for (int b = 0; b < B; ++b) x[(i + B + b) * ld] = scale * a1[b];
  }
  for (int i = nb * B; i < n; ++i) x[i * ld] *= scale;
}

constexpr int kRedThreads = 512;  // reduction kernels: 8 wavefronts with room for 256 VGPRs
// Panel kernel: 16 wavefronts (128 VGPRs each) with tiles of 3 x kRedCols loads in flight;
// more wavefronts beat deeper tiles for this latency-bound pass (measured on gfx950)
constexpr int kPanelThreads = 1024;
constexpr int kPanelChunks = 3;
constexpr int kRedCols = 4;  // columns per wavefront group in the reduction pass

__device__ inline double block_max(double v, double* red, int tid, int bs) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (bs + 63) / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// Off-diagonal entries at most this fraction of the largest diagonal entry: the matrix is
// taken as diagonal (its diagonal has residual <= sqrt(n) * 1e-13 ||A||).
constexpr double kDiagTol = 1e-13;
// A spectrum inside the disc |lambda - mu| <= kShiftTol |mu| (mu the mean diagonal entry,
// radius by Gershgorin) is computed as mu + eig(A - mu I): a Gram matrix of nearly
// orthonormal vectors then becomes an ordinary problem instead of one huge cluster.
constexpr double kShiftTol = 1e-3;
// Off-diagonal entries of T at most this multiple of eps ||T|| split T into blocks.
constexpr double kSplitTol = 4.0 * 2.220446049250313e-16;
// Neighbouring eigenvalues (both above the zero cut) closer than
// min(kClusterTol ||T||, kClusterRel max|lambda|) form a cluster whose inverse-iteration
// vectors are orthogonalised against each other.  Outside clusters a vector is accurate to
// about eps ||T|| / gap: orthogonal to ~1e-9 where |lambda| >= 1e-5 ||T||, and in the graded
// tail only as far as eps ||T|| / (0.01 |lambda|), which weighted by sqrt(|lambda|) (as in
// a Gram factor V Lambda^{1/2}) stays below ~1e-9 ||T||.
constexpr double kClusterTol = 1e-7;
constexpr double kClusterRel = 1e-2;
// Eigenvalues without a close neighbour get their vector from one thread; clusters of two or
// more go to the workgroup (one thread per member, orthogonalisation by the workgroup): a
// thread that works through a cluster alone serialises its members' solves and their strided
// orthogonalisation, which was measured to set the length of whole launches.
// Inverse-iteration solves per vector outside clusters: with an eigenvalue from
// multisection (error ~ eps ||T||) each solve shrinks the components along the other
// eigenvectors by about eps ||T|| / gap, so two solves suffice at the cluster threshold.
constexpr int kInvIters = 2;

__device__ inline bool linked(double a, double b, double cut, double ctol) {
  return fabs(a) > cut && fabs(b) > cut && b - a <= fmin(ctol, kClusterRel * fmax(fabs(a), fabs(b)));
}

__device__ inline double start_value(int i, int j) {
  return 1.0 + 0.37 * (double)((i * 7919 + j * 104729) % 101) / 101.0;
}


// Work layout of one problem (doubles): [0, n^2) working copy, reflectors below the
// diagonal; [n^2, 6 n^2) per-thread inverse-iteration storage (during the reduction: the
// current panel's vectors); [6 n^2, 7 n^2) eigenvectors of T in descending order; then beta_k,
// the diagonal d and off-diagonal e of T (n each), the applied shift, the eigenvalues of T
// in bisection order and their descending ranks (n each).

// Layout after the reduction, past the eigenvector area of T (doubles): beta_k, d, e (n
// each), the applied shift, then the eigenvalues of T in bisection order and the
// descending rank of each (n each).
__device__ inline gdouble* tri_tail(gdouble* W, int n) { return W + 7 * (int64_t)n * n; }
// 1 when the reduction found the input diagonal (T = diag(A), no reflectors); kept in the
// rank area of the tail, which the eigenvalue phase overwrites.
__device__ inline gdouble* tri_diag_flag(gdouble* W, int n) { return tri_tail(W, n) + 4 * n + 1; }

// 1. Blocked reduction to tridiagonal form (one workgroup per matrix per launch).
//
// 1a. Preparation: working copy of A (both triangles, from the upper triangle of the
//     input); a matrix whose off-diagonal part is negligible is passed on as T = diag(A);
//     a narrow spectrum is shifted by its mean diagonal entry.
//
//     The copy runs on 32 x 32 tiles of the upper triangle, many workgroups per matrix: a
//     tile is read along its columns, written in place and, through LDS, transposed into
//     the lower triangle.  Each tile also leaves the largest diagonal and off-diagonal
//     magnitudes and its share of the off-diagonal absolute row sums (the Gershgorin
//     radii): entry [b][x] of the partial sums holds what tile row or column block b
//     contributes to row x, so every entry has exactly one writer.  A second kernel, one
//     workgroup per matrix, reduces those partials and takes the decisions.
constexpr int kPrepTile = 32;
__device__ inline int prep_tiles(int n) { return (n + kPrepTile - 1) / kPrepTile; }
// partial row sums (tiles(n) x n) and the per-tile maxima (2 per tile pair), past the
// working copy in the area the later phases use as scratch
__device__ inline gdouble* prep_rowsums(gdouble* W, int n) { return W + (int64_t)n * n; }
__device__ inline gdouble* prep_maxima(gdouble* W, int n) { return prep_rowsums(W, n) + (int64_t)prep_tiles(n) * n; }

__global__ __launch_bounds__(256) void tridiag_copy_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double tile[kPrepTile][kPrepTile + 1];  // tile[c][r] = A[r, c] of the input
  __shared__ double red[2][4];
  const EigDesc D = descs[blockIdx.y];
  const int n = D.n;
  const int T = prep_tiles(n);
  const int p = blockIdx.x;
  if (n <= 0 || p >= T * (T + 1) / 2) return;
  // tile pair p -> (bi, bj), bi <= bj, p = bj (bj + 1) / 2 + bi
  int bj = int((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (bj * (bj + 1) / 2 > p) --bj;
  while ((bj + 1) * (bj + 2) / 2 <= p) ++bj;
  const int bi = p - bj * (bj + 1) / 2;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  const int r0 = bi * kPrepTile, c0 = bj * kPrepTile;
  gcdouble* Ain = gbl(D.A);
  gdouble* A = gbl(D.work);
  double dg = 0.0, od = 0.0;
#pragma unroll
  for (int q = 0; q < kPrepTile / 8; ++q) {
    const int cl = ty + 8 * q, r = r0 + tx, c = c0 + cl;
    const bool ok = r < n && c < n && r <= c;
    const double v = ok ? Ain[r + (int64_t)c * D.lda] : 0.0;
    tile[cl][tx] = v;
    if (ok) {
      A[r + (int64_t)c * n] = v;
      if (r == c) dg = fmax(dg, fabs(v)); else od = fmax(od, fabs(v));
    }
  }
  __syncthreads();
  // transposed part: A[c, r] = A[r, c] for r < c, written along c
#pragma unroll
  for (int q = 0; q < kPrepTile / 8; ++q) {
    const int rl = ty + 8 * q, r = r0 + rl, c = c0 + tx;
    if (r < n && c < n && r < c) A[c + (int64_t)r * n] = tile[tx][rl];
  }
  // off-diagonal absolute sums: column c of the tile (rows r < c) and row r (columns c > r)
  gdouble* P = prep_rowsums(A, n);
  if (tid < 2 * kPrepTile) {
    const int x = tid & 31;
    double sum = 0.0;
    if (tid < kPrepTile) {
      for (int rl = 0; rl < kPrepTile; ++rl)
        if (r0 + rl < c0 + x) sum += fabs(tile[x][rl]);
    } else {
      for (int cl = 0; cl < kPrepTile; ++cl)
        if (c0 + cl > r0 + x) sum += fabs(tile[cl][x]);
    }
    if (bi == bj) {  // both sums belong to row x of the same block
      const double other = __shfl_xor(sum, 32, 64);
      if (tid < kPrepTile && r0 + x < n) P[(int64_t)bi * n + r0 + x] = sum + other;
    } else if (tid < kPrepTile) {
      if (c0 + x < n) P[(int64_t)bi * n + c0 + x] = sum;
    } else {
      if (r0 + x < n) P[(int64_t)bj * n + r0 + x] = sum;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dg = fmax(dg, __shfl_xor(dg, off, 64));
    od = fmax(od, __shfl_xor(od, off, 64));
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = dg;
    red[1][tid >> 6] = od;
  }
  __syncthreads();
  if (tid == 0) {
    gdouble* M = prep_maxima(A, n);
    M[2 * p] = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    M[2 * p + 1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
  }
}

__global__ __launch_bounds__(kRedThreads) void tridiag_prepare_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double red[kRedThreads / 64];
  const EigDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lda = n;
  gdouble* A = gbl(D.work);
  gdouble* tail = tri_tail(A, n);
  gdouble* betas = tail;
  gdouble* dd = tail + n;
  gdouble* ee = tail + 2 * n;
  const int T = prep_tiles(n), np = T * (T + 1) / 2;
  gcdouble* P = prep_rowsums(A, n);
  gcdouble* M = prep_maxima(A, n);
  double od = 0.0, dg = 0.0;
  for (int t = tid; t < np; t += bs) {
    dg = fmax(dg, M[2 * t]);
    od = fmax(od, M[2 * t + 1]);
  }
  od = block_max(od, red, tid, bs);
  dg = block_max(dg, red, tid, bs);
  if (od <= kDiagTol * dg) {
    for (int t = tid; t < n; t += bs) {
      dd[t] = A[t + (int64_t)t * lda];
      ee[t] = 0.0;
      betas[t] = 0.0;
    }
    if (tid == 0) {
      tail[3 * n] = 0.0;
      *tri_diag_flag(A, n) = 1.0;
    }
    return;
  }
  double dsum = 0.0;
  for (int t = tid; t < n; t += bs) dsum += A[t + (int64_t)t * lda];
  const double mu = block_sum(dsum, red, tid, bs) / n;
  double rad = 0.0;
  for (int j = tid; j < n; j += bs) {
    double r = fabs(A[j + (int64_t)j * lda] - mu);
    for (int b = 0; b < T; ++b) r += P[(int64_t)b * n + j];
    rad = fmax(rad, r);
  }
  rad = block_max(rad, red, tid, bs);
  const double shift = rad <= kShiftTol * fabs(mu) ? mu : 0.0;
  if (shift != 0.0)
    for (int t = tid; t < n; t += bs) A[t + (int64_t)t * lda] -= shift;
  if (tid == 0) {
    tail[3 * n] = shift;
    *tri_diag_flag(A, n) = 0.0;
  }
}

// 1b. One panel: steps k = k0 .. k0 + nbe - 1 (nbe = min(kTriPanel, n - 2 - k0)).  Step k
//     takes column k of the matrix as updated by all earlier steps, forms the reflector
//     H_k = I - beta v v^T (v_{k+1} = 1, |v_i| <= 1, beta in [1, 2]), stores v below the
//     diagonal, and computes p = A_k v, q = beta p - (beta^2/2)(p^T v) v, so that step k's
//     update is A <- A - v q^T - q v^T.  The stored matrix only carries the updates of
//     earlier panels; within the panel
//       A_k = A_stored - sum_{j < k} (v_j q_j^T + q_j v_j^T),
//     so p is the product of the stored trailing lower triangle with v (one read-only pass:
//     a_ij adds a_ij v_i to p_j and a_ij v_j to p_i for i > j) minus the panel terms, and
//     the next column is corrected the same way.  The panel's v and q go to
//     P1 = [V | Q] and P2 = [Q | V] (n x 2 nbe each, after the working copy), from which
//     the caller applies A22 <- A22 - P1 P2^T to the trailing block (a GEMM) before the
//     next panel.
__global__ __launch_bounds__(kPanelThreads) void tridiag_panel_kernel(const EigDesc* __restrict__ descs, int k0) {
  __shared__ double red[kPanelThreads / 64];
  __shared__ double rowc[2 * kTriPanel];  // row k + 1 of the panel: Q, then V
  // v, next column, column products: n doubles each; panel dot products 2 kTriPanel;
  // nw x n per-wavefront row products
  extern __shared__ double tsm[];
  const EigDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (k0 + 2 >= n) return;
  const int nbe = min(kTriPanel, n - 2 - k0);
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
  const int lda = n;
  const int64_t nn0 = (int64_t)n * n;
  gdouble* A = gbl(D.work);
  gdouble* tail = tri_tail(A, n);
  gdouble* betas = tail;
  gdouble* dd = tail + n;
  gdouble* ee = tail + 2 * n;
  gdouble* P1 = A + nn0;
  gdouble* P2 = P1 + (int64_t)2 * nbe * n;
  if (*tri_diag_flag(A, n) != 0.0) {  // nothing to reduce: the trailing update is zero
    for (int64_t e = tid; e < (int64_t)4 * nbe * n; e += bs) P1[e] = 0.0;
    return;
  }
  double* vk = tsm;
  double* nxt = vk + n;
  double* pd = nxt + n;
  double* xw = pd + n;
  double* xv = xw + kTriPanel;
  double* pw = xv + kTriPanel;
  // column k0 as left by the earlier panels; row i is owned by thread i mod bs throughout
  for (int i = tid; i < n; i += bs) nxt[i] = i >= k0 ? A[i + (int64_t)k0 * lda] : 0.0;
  for (int j = 0; j < nbe; ++j) {
    const int k = k0 + j;
    double part = 0.0;
    for (int i = tid; i < n; i += bs)
      if (i >= k + 2) part += nxt[i] * nxt[i];
    const double sig2 = block_sum(part, red, tid, bs);  // also publishes nxt
    const double x0 = nxt[k + 1], akk = nxt[k];
    double beta = 0.0, alpha = x0, inv = 0.0;
    if (sig2 != 0.0) {
      const double nrm = sqrt(x0 * x0 + sig2);
      alpha = x0 > 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;  // |v0| >= nrm
      beta = 2.0 * v0 * v0 / (v0 * v0 + sig2);
      inv = 1.0 / v0;
    }
    if (tid == 0) {
      ee[k] = alpha;
      dd[k] = akk;
      betas[k] = beta;
    }
    gdouble* Vj = P1 + (int64_t)j * n;
    gdouble* Qj = P1 + (int64_t)(nbe + j) * n;
    gdouble* Qj2 = P2 + (int64_t)j * n;
    gdouble* Vj2 = P2 + (int64_t)(nbe + j) * n;
    for (int i = tid; i < n; i += bs) {
      const double v = (beta == 0.0 || i <= k) ? 0.0 : (i == k + 1 ? 1.0 : nxt[i] * inv);
      vk[i] = v;
      if (beta != 0.0 && i > k) A[i + (int64_t)k * lda] = v;  // v stored below the diagonal
      Vj[i] = v;
      Vj2[i] = v;
    }
    __syncthreads();
    // dot products of v with the panel's earlier vectors (rows > k)
    if (tid < j) {
      rowc[tid] = P1[k + 1 + (int64_t)(nbe + tid) * n];
      rowc[kTriPanel + tid] = P1[k + 1 + (int64_t)tid * n];
    }
    for (int jj = wave; jj < j; jj += nw) {
      gcdouble* Vc = P1 + (int64_t)jj * n;
      gcdouble* Qc = P1 + (int64_t)(nbe + jj) * n;
      double a = 0.0, b = 0.0;
      // the loads of a 256-row pass are issued before they are used (addresses clamped)
      for (int i0 = k + 1; i0 < n; i0 += 256) {
        double qa[4], va[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ic = min(i0 + 64 * u + lane, n - 1);
          qa[u] = Qc[ic];
          va[u] = Vc[ic];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 64 * u + lane;
          const double vi = i < n ? vk[i] : 0.0;
          a += qa[u] * vi;
          b += va[u] * vi;
        }
      }
      a = wave_sum_d(a);
      b = wave_sum_d(b);
      if (lane == 0) {
        xw[jj] = a;
        xv[jj] = b;
      }
    }
    // read-only pass over the stored trailing lower triangle: wavefront w takes columns
    // k + 1 + w + nw c in groups of kRedCols, rows in tiles of kPanelChunks 64-row chunks,
    // the next tile's loads issued before the current one is consumed; a_ij v_j terms go
    // to the wavefront's own LDS row pw[w] (in order within the wavefront)
    double* pwr = pw + wave * n;
    for (int i = k + 1 + lane; i < n; i += 64) pwr[i] = 0.0;
    const int64_t cstep = (int64_t)nw * lda;
    int j0 = k + 1 + wave, i0 = j0;
    double cur[kPanelChunks][kRedCols];
    auto load_tile = [&](double (&t)[kPanelChunks][kRedCols], int tj0, int ti0) {
      gcdouble* colj = A + (int64_t)tj0 * lda;
#pragma unroll
      for (int h = 0; h < kPanelChunks; ++h) {
        const int i = ti0 + 64 * h + lane;
#pragma unroll
        for (int c = 0; c < kRedCols; ++c) t[h][c] = (i < n && i >= tj0 + c * nw) ? colj[i + c * cstep] : 0.0;
      }
    };
    double vj[kRedCols], dot[kRedCols];
    auto start_group = [&](int tj0) {
#pragma unroll
      for (int c = 0; c < kRedCols; ++c) {
        const int jc = tj0 + c * nw;
        vj[c] = jc < n ? vk[jc] : 0.0;
        dot[c] = 0.0;
      }
    };
    if (j0 < n) {
      start_group(j0);
      load_tile(cur, j0, i0);
    }
    while (j0 < n) {
      int nj0 = j0, ni0 = i0 + 64 * kPanelChunks;
      if (ni0 >= n) { nj0 = j0 + kRedCols * nw; ni0 = nj0; }
      double nxtt[kPanelChunks][kRedCols];
      if (nj0 < n) load_tile(nxtt, nj0, ni0);
#pragma unroll
      for (int h = 0; h < kPanelChunks; ++h) {
        const int i = i0 + 64 * h + lane;
        if (i >= n) continue;
        const double vki = vk[i];
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kRedCols; ++c) {
          const int jc = j0 + c * nw;
          const double x = cur[h][c];  // zero outside the triangle
          dot[c] += x * vki;
          if (i > jc) acc += x * vj[c];
        }
        pwr[i] += acc;
      }
      if (nj0 != j0) {  // group finished
#pragma unroll
        for (int c = 0; c < kRedCols; ++c) {
          const double d = wave_sum_d(dot[c]);
          if (lane == 0 && j0 + c * nw < n) pd[j0 + c * nw] = d;
        }
        if (nj0 < n) start_group(nj0);
      }
#pragma unroll
      for (int h = 0; h < kPanelChunks; ++h)
#pragma unroll
        for (int c = 0; c < kRedCols; ++c) cur[h][c] = nxtt[h][c];
      j0 = nj0;
      i0 = ni0;
    }
    __syncthreads();
    // p = A_k v (beta p kept in pd), and the panel terms of the next column
    const bool more = j + 1 < nbe;
    double pv = 0.0;
    for (int i = tid; i < n; i += bs) {
      if (i <= k) continue;
      double p = pd[i];
      for (int w2 = 0; w2 < nw; ++w2) p += pw[w2 * n + i];
      double cn = 0.0;
      // panel terms in groups of 4 columns, each group's loads issued first
      for (int jb = 0; jb < j; jb += 4) {
        double va[4], qa[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = min(jb + u, j - 1);
          va[u] = P1[i + (int64_t)jj * n];
          qa[u] = P1[i + (int64_t)(nbe + jj) * n];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (jb + u >= j) break;
          const int jj = jb + u;
          p -= va[u] * xw[jj] + qa[u] * xv[jj];
          cn += va[u] * rowc[jj] + qa[u] * rowc[kTriPanel + jj];
        }
      }
      p *= beta;
      pd[i] = p;
      if (more) nxt[i] = cn;
      pv += p * vk[i];
    }
    const double vtp = block_sum(pv, red, tid, bs);  // also publishes pd
    const double K = 0.5 * beta * vtp;
    const double q1 = pd[k + 1] - K * vk[k + 1];
    for (int i = tid; i < n; i += bs) {
      const double q = i <= k ? 0.0 : pd[i] - K * vk[i];
      Qj[i] = q;
      Qj2[i] = q;
      // column k + 1 after step k, rows >= k + 1
      if (more && i > k) nxt[i] = A[i + (int64_t)(k + 1) * lda] - nxt[i] - vk[i] * q1 - q * vk[k + 1];
    }
  }
}

// 1b'. The same reduction one step per launch, G workgroups per problem (for batches of
//     few problems, where one workgroup per matrix leaves most compute units idle).  The
//     full symmetric working copy is updated every step; workgroup g of a problem owns the
//     columns j = g (mod G), so a column stays with one workgroup (and one XCD's L2) for
//     the whole reduction.  Launch k (k = 0 .. n - 2):
//       - every workgroup reads p_{k-1} (= beta_{k-1} A^(k-1) v_{k-1}) and v_{k-1} and
//         forms q_{k-1} = p_{k-1} - (beta_{k-1}/2)(p_{k-1}^T v_{k-1}) v_{k-1};
//       - it forms column k of A^(k) = A^(k-1) - v_{k-1} q_{k-1}^T - q_{k-1} v_{k-1}^T from
//         the stored column k (which holds A^(k-1)) and from it the reflector v_k, beta_k
//         (the same arithmetic in every workgroup, so every copy agrees bit for bit);
//       - on its own columns j >= k + 1 (rows >= k + 1) it applies step k - 1's update,
//         stores the result and takes p_k[j] = beta_k (column j)^T v_k, which by symmetry is
//         entry j of beta_k A^(k) v_k: no reduction across workgroups is needed, the launch
//         boundary is the only synchronisation.
//     Workgroup 0 records d_k, e_k, beta_k and v_k, and moves v_{k-1} below the diagonal of
//     column k - 1 (which no workgroup reads in launch k).  Launch n - 2 applies the last
//     update to the final 2 x 2 block and records it.  Both products of the rank-2 update
//     are rounded before they are added, so the updated copy stays exactly symmetric.
//     p and v alternate between two n-vectors by the parity of k, after the working copy.
constexpr int kStepThreads = 256;
static_assert(kStepThreads % 64 == 0 && kEigMax % kStepThreads == 0, "step kernel layout");

__device__ inline double sym_rank2(double vi, double qj, double qi, double vj) {
#pragma clang fp contract(off)
  return vi * qj + qi * vj;
}

// rows r0 .. n - 1 of a column, lane-strided 64-row chunks (zero past the end)
template <int CH>
__device__ inline void step_load_col(gcdouble* col, int r0, int n, int lane, double (&a)[CH]) {
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    const int i = r0 + 64 * u + lane;
    a[u] = i < n ? col[i] : 0.0;
  }
}

// Each launch is latency bound (a few hundred rows per problem and step), so every load
// that does not depend on the step's own results is issued at the start: the first own
// column of each wavefront, and p_{k-1}, v_{k-1} and column k (at most kStepVec rows per
// thread); the next own column is loaded while the current one is processed.  CH 64-row
// chunks cover a column (n <= 64 CH), VEC = CH / 4 rows per thread the column-k pass; the
// smaller instances hold fewer registers and so keep more wavefronts per compute unit.
template <int CH>
__global__ __launch_bounds__(kStepThreads) void tridiag_step_kernel(const EigDesc* __restrict__ descs, int k,
                                                                    int G) {
  constexpr int kStepChunks = CH;
  constexpr int kStepVec = CH * 64 / kStepThreads;
  static_assert(kStepVec >= 1 && kStepVec * kStepThreads == 64 * CH, "step kernel instance");
  __shared__ double red[kStepThreads / 64];
  __shared__ double vprev[64 * CH], qprev[64 * CH], vcur[64 * CH];
  const int prob = blockIdx.x / G, g = blockIdx.x - prob * G;
  const EigDesc D = descs[prob];
  const int n = D.n;
  if (n <= 0 || n > 64 * CH || k > max(n - 2, 0)) return;
  gdouble* A = gbl(D.work);
  if (*tri_diag_flag(A, n) != 0.0) return;
  const int tid = threadIdx.x, bs = kStepThreads;
  const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
  const int64_t lda = n;
  gdouble* tail = tri_tail(A, n);
  gdouble* betas = tail;
  gdouble* dd = tail + n;
  gdouble* ee = tail + 2 * n;
  gdouble* pbuf = A + (int64_t)n * n;
  gdouble* vbuf = pbuf + 2 * lda;
  if (n == 1) {
    if (g == 0 && tid == 0) {
      dd[0] = A[0];
      ee[0] = 0.0;
      betas[0] = 0.0;
    }
    return;
  }
  const bool upd = k > 0;
  // first own column of this wavefront (columns j = g mod G, j >= k + 1)
  int j = k + 1 + ((g - (k + 1)) % G + G) % G + wave * G;
  double cur[kStepChunks];
  if (j < n) step_load_col(A + (int64_t)j * lda, k + 1, n, lane, cur);
  gcdouble* pp = pbuf + (int64_t)((k + 1) & 1) * lda;  // step k - 1's vectors
  gcdouble* vp = vbuf + (int64_t)((k + 1) & 1) * lda;
  double pv[kStepVec], vv[kStepVec], ck[kStepVec];
#pragma unroll
  for (int u = 0; u < kStepVec; ++u) {
    const int i = k + tid + u * bs;
    const bool in = i < n;
    pv[u] = upd && in ? pp[i] : 0.0;
    vv[u] = upd && in ? vp[i] : 0.0;
    ck[u] = in ? A[i + (int64_t)k * lda] : 0.0;
  }
  const double bprev = upd ? betas[k - 1] : 0.0;
  // q_{k-1} = p_{k-1} - (beta_{k-1}/2)(p_{k-1}^T v_{k-1}) v_{k-1}  (p carries beta)
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < kStepVec; ++u) part += pv[u] * vv[u];
  const double K = 0.5 * bprev * block_sum(part, red, tid, bs);
  double qq[kStepVec];
#pragma unroll
  for (int u = 0; u < kStepVec; ++u) {
    const int i = k + tid + u * bs;
    qq[u] = pv[u] - K * vv[u];
    if (i < n) {
      vprev[i] = vv[u];
      qprev[i] = qq[u];
    }
  }
  __syncthreads();
  // v_{k-1} goes below the diagonal of column k - 1 for the back-transformation
  if (g == 0 && bprev != 0.0) {
#pragma unroll
    for (int u = 0; u < kStepVec; ++u) {
      const int i = k + tid + u * bs;
      if (i < n) A[i + (int64_t)(k - 1) * lda] = vv[u];
    }
  }
  // column k of A^(k), rows k .. n - 1
  const double qk = qprev[k], vk = vprev[k];
  part = 0.0;
#pragma unroll
  for (int u = 0; u < kStepVec; ++u) {
    const int i = k + tid + u * bs;
    if (upd) ck[u] -= sym_rank2(vv[u], qk, qq[u], vk);
    if (i < n) vcur[i] = ck[u];
    if (i >= k + 2 && i < n) part += ck[u] * ck[u];
  }
  const double sig2 = block_sum(part, red, tid, bs);  // also publishes vcur
  if (k == n - 2) {  // the final 2 x 2 block
    if (g == 0 && tid == 0) {
      double a = A[(n - 1) + (int64_t)(n - 1) * lda];
      if (upd) a -= sym_rank2(vprev[n - 1], qprev[n - 1], qprev[n - 1], vprev[n - 1]);
      dd[n - 2] = vcur[n - 2];
      ee[n - 2] = vcur[n - 1];
      betas[n - 2] = 0.0;
      dd[n - 1] = a;
      ee[n - 1] = 0.0;
      betas[n - 1] = 0.0;
    }
    return;
  }
  // reflector H_k = I - beta v v^T with v_{k+1} = 1 mapping column k below the diagonal
  // onto alpha e_{k+1}
  const double x0 = vcur[k + 1], akk = vcur[k];
  double beta = 0.0, alpha = x0, inv = 0.0;
  if (sig2 != 0.0) {
    const double nrm = sqrt(x0 * x0 + sig2);
    alpha = x0 > 0.0 ? -nrm : nrm;
    const double v0 = x0 - alpha;
    beta = 2.0 * v0 * v0 / (v0 * v0 + sig2);
    inv = 1.0 / v0;
  }
  __syncthreads();  // every thread has read x0 and akk before vcur becomes v
  gdouble* vout = vbuf + (int64_t)(k & 1) * lda;
  gdouble* pout = pbuf + (int64_t)(k & 1) * lda;
#pragma unroll
  for (int u = 0; u < kStepVec; ++u) {
    const int i = k + tid + u * bs;
    if (i >= n) continue;
    const double v = (beta == 0.0 || i == k) ? 0.0 : (i == k + 1 ? 1.0 : ck[u] * inv);
    vcur[i] = v;
    if (g == 0) vout[i] = v;
  }
  if (g == 0 && tid == 0) {
    ee[k] = alpha;
    dd[k] = akk;
    betas[k] = beta;
  }
  __syncthreads();
  // own columns j >= k + 1: step k - 1's update, then p_k[j] = beta_k (column j)^T v_k
  while (j < n) {
    const int jn = j + nw * G;
    double nxt[kStepChunks];
    if (jn < n) step_load_col(A + (int64_t)jn * lda, k + 1, n, lane, nxt);
    gdouble* col = A + (int64_t)j * lda;
    const double qj = qprev[j], vj = vprev[j];
    double dot = 0.0;
#pragma unroll
    for (int u = 0; u < kStepChunks; ++u) {
      const int i = k + 1 + 64 * u + lane;
      if (i >= n) continue;
      double a = cur[u];
      if (upd) {
        a -= sym_rank2(vprev[i], qj, qprev[i], vj);
        col[i] = a;
      }
      dot += a * vcur[i];
    }
    dot = wave_sum_d(dot);
    if (lane == 0) pout[j] = beta * dot;
#pragma unroll
    for (int u = 0; u < kStepChunks; ++u) cur[u] = nxt[u];
    j = jn;
  }
}

// 1b''. The last steps of the step-per-launch reduction, one workgroup per problem with the
//      trailing block (at most kTailMax rows) held in registers, where a step costs four
//      workgroup barriers instead of a launch.  Entered at k0 = max(n - kTailMax, 0): the
//      stored columns >= k0 hold A^(k0-1), and for k0 > 0 step k0 - 1's p and v wait in the
//      alternating vectors, as the step kernel leaves them.  Steps k0 .. n - 3 then run as
//      in the step kernel (same reflector, same symmetric rank-2 form, but every update is
//      applied at once), and the final 2 x 2 block is recorded.  Wave w owns the columns
//      j = w (mod waves), lane l the rows l, l + 64, l + 128 of them (kTailCols x kTailRows
//      values per lane): the wave forms their partial products with v along the rows
//      (summed over the waves through LDS, so no cross-lane reductions), updates them, and
//      the owner of the next reflector's column leaves it and its squared norm in LDS for
//      the next step.  Every step runs over the whole block: v and p are zero outside the
//      active rows, which leaves the finished rows and columns unchanged.
constexpr int kTailMax = 192;
constexpr int kTailThreads = 1024;
constexpr int kTailWaves = kTailThreads / 64;
constexpr int kTailCols = kTailMax / kTailWaves;  // columns per wavefront
constexpr int kTailRows = kTailMax / 64;          // rows per lane and column
static_assert(kTailCols * kTailWaves == kTailMax && kTailRows * 64 == kTailMax, "tail layout");

__global__ __launch_bounds__(kTailThreads) void tridiag_tail_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double part[kTailWaves * kTailMax];  // row partials of A v, one row of kTailMax per wave
  // xsh/sh_sig2: the next reflector's column and its squared norm below the subdiagonal,
  // in two buffers by the parity of the step (read in step c, written for step c + 1)
  __shared__ double vsh[kTailMax], psh[kTailMax], xsh[2][kTailMax], red[kTailWaves];
  __shared__ double sh_sig2[2];
  const EigDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (n <= 0) return;
  gdouble* A = gbl(D.work);
  if (*tri_diag_flag(A, n) != 0.0) return;
  const int tid = threadIdx.x, bs = kTailThreads;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t lda = n;
  gdouble* tail = tri_tail(A, n);
  gdouble* betas = tail;
  gdouble* dd = tail + n;
  gdouble* ee = tail + 2 * n;
  if (n == 1) {
    if (tid == 0) {
      dd[0] = A[0];
      ee[0] = 0.0;
      betas[0] = 0.0;
    }
    return;
  }
  const int k0 = max(n - kTailMax, 0), m0 = n - k0;
  for (int i = tid; i < kTailMax; i += bs) {
    vsh[i] = 0.0;
    psh[i] = 0.0;
  }
  __syncthreads();
  // pending update of step k0 - 1: v in vsh, q = p - (beta/2)(p^T v) v in psh (local rows)
  if (k0 > 0) {
    gcdouble* pp = A + (int64_t)n * n + (int64_t)((k0 - 1) & 1) * lda;
    gcdouble* vp = A + (int64_t)n * n + 2 * lda + (int64_t)((k0 - 1) & 1) * lda;
    const double bprev = betas[k0 - 1];
    double pv = 0.0;
    for (int i = tid; i < m0; i += bs) {
      const double v = vp[k0 + i], p = pp[k0 + i];
      vsh[i] = v;
      psh[i] = p;
      pv += p * v;
    }
    const double K = 0.5 * bprev * block_sum(pv, red, tid, bs);
    for (int i = tid; i < m0; i += bs) psh[i] -= K * vsh[i];
    __syncthreads();
    if (bprev != 0.0)
      for (int i = tid; i < m0; i += bs) A[(k0 + i) + (int64_t)(k0 - 1) * lda] = vsh[i];
  }
  // the block into registers (zero outside it), with the pending update applied; the owner
  // of column 0 publishes it and its squared norm below the subdiagonal entry
  double a[kTailCols][kTailRows];
#pragma unroll
  for (int t = 0; t < kTailCols; ++t) {
    const int j = wave + kTailWaves * t;
    const double qj = psh[j], vj = vsh[j];
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < kTailRows; ++r) {
      const int i = lane + 64 * r;
      double x = 0.0;
      if (i < m0 && j < m0) {
        x = A[(k0 + i) + (int64_t)(k0 + j) * lda];
        if (k0 > 0) x -= sym_rank2(vsh[i], qj, psh[i], vj);
      }
      a[t][r] = x;
      if (j == 0) {
        xsh[0][i] = x;
        if (i >= 2) sq += x * x;
      }
    }
    if (j == 0) {
      sq = wave_sum_d(sq);
      if (lane == 0) sh_sig2[0] = sq;
    }
  }
  __syncthreads();
  for (int c = 0; k0 + c + 2 < n; ++c) {
    const int k = k0 + c;
    // reflector of column c below the diagonal, formed by every thread from column c
    // (published before the last barrier)
    const int b = c & 1;
    const double sig2 = sh_sig2[b];
    const double x0 = xsh[b][c + 1];
    double beta = 0.0, alpha = x0, inv = 0.0;
    if (sig2 != 0.0) {
      const double nrm = sqrt(x0 * x0 + sig2);
      alpha = x0 > 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      beta = 2.0 * v0 * v0 / (v0 * v0 + sig2);
      inv = 1.0 / v0;
    }
    auto vof = [&](int i) {
      return (beta == 0.0 || i <= c || i >= m0) ? 0.0 : (i == c + 1 ? 1.0 : xsh[b][i] * inv);
    };
    if (tid == 0) {
      ee[k] = alpha;
      dd[k] = xsh[b][c];
      betas[k] = beta;
    }
    if (beta != 0.0)
      for (int i = c + 1 + tid; i < m0; i += bs) A[(k0 + i) + (int64_t)k * lda] = vof(i);  // below the diagonal of column k
    double vr[kTailRows];
#pragma unroll
    for (int r = 0; r < kTailRows; ++r) vr[r] = vof(lane + 64 * r);
    const int nxt = c + 1;  // the next reflector's column
    double K = 0.0;
    if (beta != 0.0) {
      // row partials of A22 v over each wavefront's columns, then p = beta A22 v
      double acc[kTailRows] = {};
#pragma unroll
      for (int t = 0; t < kTailCols; ++t) {
        const int j = wave + kTailWaves * t;
        if (j <= c || j >= m0) continue;
        const double vj = vof(j);
#pragma unroll
        for (int r = 0; r < kTailRows; ++r) acc[r] += a[t][r] * vj;
      }
#pragma unroll
      for (int r = 0; r < kTailRows; ++r) {
        if (64 * r + 63 <= c || 64 * r >= m0) continue;  // a chunk of finished (or absent) rows
        part[wave * kTailMax + lane + 64 * r] = acc[r];
      }
      __syncthreads();
      for (int i = tid; i < kTailMax; i += bs) {
        double p = 0.0;
        if (i > c && i < m0) {
#pragma unroll 4
          for (int w = 0; w < kTailWaves; ++w) p += part[w * kTailMax + i];
          p *= beta;
        }
        psh[i] = p;
      }
      __syncthreads();
      // K = (beta/2) p^T v (every wavefront forms it)
      double pv = 0.0;
#pragma unroll
      for (int r = 0; r < kTailRows; ++r) pv += psh[lane + 64 * r] * vr[r];
      K = 0.5 * beta * wave_sum_d(pv);
    }
    // q = p - K v and the rank-2 update of the own columns (the identity when beta = 0);
    // the owner of column nxt publishes it
#pragma unroll
    for (int t = 0; t < kTailCols; ++t) {
      const int j = wave + kTailWaves * t;
      if (j <= c || j >= m0) continue;  // finished (or absent) columns stay as they are
      double sq = 0.0;
      if (beta != 0.0) {
        const double vj = vof(j), qj = psh[j] - K * vj;
#pragma unroll
        for (int r = 0; r < kTailRows; ++r) {
          if (64 * r + 63 <= c || 64 * r >= m0) continue;
          const double qi = psh[lane + 64 * r] - K * vr[r];
          a[t][r] -= sym_rank2(vr[r], qj, qi, vj);
        }
      }
      if (j == nxt) {
#pragma unroll
        for (int r = 0; r < kTailRows; ++r) {
          if (64 * r + 63 <= c || 64 * r >= m0) continue;
          const int i = lane + 64 * r;
          xsh[b ^ 1][i] = a[t][r];
          if (i >= nxt + 2) sq += a[t][r] * a[t][r];
        }
        sq = wave_sum_d(sq);
        if (lane == 0) sh_sig2[b ^ 1] = sq;
      }
    }
    __syncthreads();
  }
  // the final 2 x 2 block: column m0 - 2 is in xsh, entry (m0 - 1, m0 - 1) with its owner
  if (tid == 0) {
    const int c = m0 - 2;
    dd[n - 2] = xsh[c & 1][c];
    ee[n - 2] = xsh[c & 1][c + 1];
    ee[n - 1] = 0.0;
    betas[n - 2] = 0.0;
    betas[n - 1] = 0.0;
  }
#pragma unroll
  for (int t = 0; t < kTailCols; ++t)
#pragma unroll
    for (int r = 0; r < kTailRows; ++r)
      if (wave + kTailWaves * t == m0 - 1 && lane + 64 * r == m0 - 1) dd[n - 1] = a[t][r];
}

// 1c. Last 2 x 2 block (or the single entry) of T, after the last trailing update.
__global__ void tridiag_finish_kernel(const EigDesc* __restrict__ descs, int nprob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob) return;
  const EigDesc D = descs[p];
  const int n = D.n;
  if (n <= 0) return;
  gdouble* A = gbl(D.work);
  if (*tri_diag_flag(A, n) != 0.0) return;
  gdouble* tail = tri_tail(A, n);
  gdouble* betas = tail;
  gdouble* dd = tail + n;
  gdouble* ee = tail + 2 * n;
  if (n >= 2) {
    dd[n - 2] = A[(n - 2) + (int64_t)(n - 2) * n];
    ee[n - 2] = A[(n - 1) + (int64_t)(n - 2) * n];
    betas[n - 2] = 0.0;
  }
  dd[n - 1] = A[(n - 1) + (int64_t)(n - 1) * n];
  ee[n - 1] = 0.0;
  betas[n - 1] = 0.0;
}


// Load d, e of T into LDS, bound ||T|| (Gershgorin) and split T at negligible off-diagonal
// entries into unreduced blocks (starts in bstart, count returned); e2 = e^2.
__device__ int tri_blocks(const EigDesc& D, int n, double* dd, double* ee, double* e2, int* bstart, int* sh_nblk,
                          double* tn_out) {
  const int tid = threadIdx.x, bs = blockDim.x;
  gcdouble* gd = tri_tail(gbl(D.work), n) + n;
  for (int i = tid; i < n; i += bs) {
    dd[i] = gd[i];
    ee[i] = gd[n + i];
  }
  __syncthreads();
  // ||T||_inf: a maximum, so the order of the partial maxima does not matter
  __shared__ double red_tn[64];
  double tn = 0.0;
  for (int i = tid; i < n; i += bs)
    tn = fmax(tn, fabs(dd[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0));
  tn = block_max(tn, red_tn, tid, bs);
  // split points in increasing order: the first wavefront takes 64 off-diagonals at a time
  // and places the split ones by the rank of their lane in the ballot
  if (tid < 64) {
    int nb = 1;
    if (tid == 0) bstart[0] = 0;
    for (int i0 = 0; i0 + 1 < n; i0 += 64) {
      const int i = i0 + tid;
      const bool sp = i + 1 < n && fabs(ee[i]) <= kSplitTol * tn;
      const unsigned long long mask = __ballot(sp);
      if (sp) {
        ee[i] = 0.0;
        bstart[nb + __popcll(mask & ((1ull << tid) - 1ull))] = i + 1;
      }
      nb += __popcll(mask);
    }
    if (tid == 0) {
      bstart[nb] = n;
      *sh_nblk = nb;
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += bs) e2[i] = ee[i] * ee[i];
  __syncthreads();
  *tn_out = tn;
  return *sh_nblk;
}

// 2. Eigenvalues of T by multisection: gridDim.x workgroups per matrix (blockIdx.y), each
//    taking one contiguous range of positions, one group of kSectLanes lanes per position;
//    position t of block b = [s, s+m) holds the (t-s)-th smallest eigenvalue of that block.
//    The bracket [a, b) keeps count(a) <= t-s < count(b); each round moves b to the first
//    of the kSectQ points whose count exceeds t-s and a to the point before it.  Every lane
//    of a group computes the same points from the same bracket, so the group stays in step.
//    The unshifted values go to the work area.
template <int LANES>
__global__ __launch_bounds__(kValuesThreads) void tridiag_values_kernel(const EigDesc* __restrict__ descs) {
  static_assert(64 % LANES == 0, "a multisection group lies within one wavefront");
  constexpr int kQ = LANES * kSectPoints;
  constexpr int kPositions = kValuesThreads / LANES;
  __shared__ int sh_nblk;
  // d, e, e2: n doubles each; block starts: n + 1 ints
  extern __shared__ double tsm[];
  const EigDesc D = descs[blockIdx.y];
  const int n = D.n;
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int t0 = blockIdx.x * chunk, t1 = min(n, t0 + chunk);
  if (n <= 0 || t0 >= t1) return;
  double* dd = tsm;
  double* ee = dd + n;
  double* e2 = ee + n;
  int* bstart = reinterpret_cast<int*>(e2 + n);
  gdouble* glam = tri_tail(gbl(D.work), n) + 3 * n + 1;
  double tn = 0.0;
  const int nblk = tri_blocks(D, n, dd, ee, e2, bstart, &sh_nblk, &tn);
  const double tiny = fmax(tn * 1e-300, 1e-300) + tn * 2.2e-16 * 1e-3;
  const int sub = threadIdx.x % LANES, grp = threadIdx.x / LANES;
  const int gbase = (threadIdx.x & 63) - sub;  // first lane of the group in its wavefront
  constexpr uint64_t kGroupMask = LANES == 64 ? ~0ull : (1ull << LANES) - 1;
  for (int t = t0 + grp; t < t1; t += kPositions) {
    int lo_b = 0, hi_b = nblk - 1;
    while (lo_b < hi_b) {
      const int mid = (lo_b + hi_b + 1) >> 1;
      if (bstart[mid] <= t) lo_b = mid; else hi_b = mid - 1;
    }
    const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
    if (m == 1) {
      if (sub == 0) glam[t] = dd[s];
      continue;
    }
    // Gershgorin interval of the block: the group's lanes take every LANES-th row and
    // combine their minima and maxima (exact in any order)
    double lo = 1e300, hi = -1e300;
    for (int i = s + sub; i < s + m; i += LANES) {
      const double r = (i > s ? fabs(ee[i - 1]) : 0.0) + (i < s + m - 1 ? fabs(ee[i]) : 0.0);
      lo = fmin(lo, dd[i] - r);
      hi = fmax(hi, dd[i] + r);
    }
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off, 64));
      hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    double a = lo - 1e-14 * tn - 1e-300, b = hi + 1e-14 * tn + 1e-300;
    const int target = t - s;
    for (int it = 0; it < 100; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (b - a <= 2.2e-16 * fmax(fabs(a), fabs(b)) * 2.0 || b - a <= 1e-18 * tn) break;
      const double h = (b - a) * (1.0 / (kQ + 1));
      auto point = [&](int j) { return fmin(fmax(a + (j + 1) * h, a), b); };
      double x[kSectPoints];
      int cnt[kSectPoints];
#pragma unroll
      for (int p = 0; p < kSectPoints; ++p) x[p] = point(sub * kSectPoints + p);
      sturm_counts<kSectPoints>(dd + s, e2 + s, m, x, tiny + 1e-300, cnt);
      int first = kSectPoints;  // this lane's first point above the target count
#pragma unroll
      for (int p = kSectPoints - 1; p >= 0; --p)
        if (cnt[p] > target) first = p;
      const uint64_t above = (__ballot(first < kSectPoints) >> gbase) & kGroupMask;
      if (above == 0) {
        a = point(kQ - 1);
      } else {
        const int l = __builtin_ctzll(above);
        const int j = l * kSectPoints + __shfl(first, gbase + l, 64);
        const double na = j > 0 ? point(j - 1) : a;
        b = point(j);
        a = na;
      }
    }
    if (sub == 0) glam[t] = 0.5 * (a + b);
  }
}

// 2b. Descending ranks of the eigenvalues, the output w (eigenvalues plus the shift, in
//     descending order; ties: lower position first) and the cut below which eigenvectors
//     are returned as zero; one workgroup per matrix.
__global__ __launch_bounds__(kTriThreads) void tridiag_rank_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double red[kTriThreads / 64];
  extern __shared__ double tsm[];  // n shifted eigenvalues
  const EigDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  gdouble* tail = tri_tail(gbl(D.work), n);
  const double shift = tail[3 * n];
  gdouble* glam = tail + 3 * n + 1;
  gdouble* grank = glam + n;
  gdouble* wout = gbl(D.w);
  double* lam = tsm;
  double mx = 0.0;
  for (int i = tid; i < n; i += bs) {
    lam[i] = glam[i] + shift;
    mx = fmax(mx, fabs(lam[i]));
  }
  mx = block_max(mx, red, tid, bs);  // also publishes lam
  if (tid == 0) tail[5 * n + 1] = D.abs_tol * mx;
  for (int t = tid; t < n; t += bs) {
    const double lt = lam[t];
    int rank = 0;
    for (int u = 0; u < n; ++u) rank += (lam[u] > lt) || (lam[u] == lt && u < t);
    grank[t] = rank;
    wout[rank] = lt;
  }
}

// 3. Eigenvectors of T by inverse iteration for the eigenvalues of descending rank below
//    nvec (all when nvec < 0): gridDim.x workgroups per matrix (blockIdx.y), each taking
//    the clusters that start in its range of positions; the vectors are left transposed in
//    V, and tridiag_sort_kernel orders them.
__global__ __launch_bounds__(kVectorPositions) void tridiag_vec_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double red[kTriThreads / 64];
  __shared__ int sh_nblk, sh_nruns;
  // d, e, e2, lam, vsh, psh, rank: n doubles each; block starts: n + 1 ints
  extern __shared__ double tsm[];
  const EigDesc D = descs[blockIdx.y];
  const int n = D.n;
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int t0 = blockIdx.x * chunk, t1 = min(n, t0 + chunk);
  if (n <= 0 || t0 >= t1) return;
  const int nvec = D.nvec < 0 ? n : min(D.nvec, n);
  if (nvec == 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
  const int64_t nn0 = (int64_t)n * n;
  double* dd = tsm;
  double* ee = dd + n;
  double* e2 = ee + n;
  double* lam = e2 + n;
  double* vsh = lam + n;
  double* psh = vsh + n;
  double* rk = psh + n;
  int* bstart = reinterpret_cast<int*>(rk + n);
  int* runs = bstart + n + 1;  // workgroup clusters: (first, last, block), at most n/2 of them
  gdouble* W = gbl(D.work);
  gdouble* scratch = W + nn0;  // per-thread inverse-iteration storage
  // eigenvectors of T, stored transposed (element i of vector t at Z[i * n + t]) so that
  // threads working on neighbouring vectors touch neighbouring addresses
  gdouble* Z = gbl(D.V);
  gcdouble* tail = tri_tail(W, n);
  const double shift = tail[3 * n];
  for (int i = tid; i < n; i += bs) {
    lam[i] = tail[3 * n + 1 + i];
    rk[i] = tail[4 * n + 1 + i];
  }
  double tn = 0.0;
  const int nblk = tri_blocks(D, n, dd, ee, e2, bstart, &sh_nblk, &tn);
  (void)e2;
  // 3. inverse iteration within each block; vectors vanish outside their block
  double lmax = 0.0;
  for (int i = tid; i < n; i += bs) lmax = fmax(lmax, fabs(lam[i]));
  lmax = block_max(lmax, red, tid, bs);
  // with a shift every |eigenvalue| of A is at least (1 - kShiftTol) |mu|: nothing is cut
  const double cut = shift != 0.0 ? 0.0 : D.abs_tol * lmax;
  const double ctol = kClusterTol * fmax(tn, 1e-300);
  const int64_t ld = n;
  const int64_t nn = (int64_t)n * n;
  for (int t = t0 + tid; t < t1; t += bs) {
    int lo_b = 0, hi_b = nblk - 1;
    while (lo_b < hi_b) {
      const int mid = (lo_b + hi_b + 1) >> 1;
      if (bstart[mid] <= t) lo_b = mid; else hi_b = mid - 1;
    }
    const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
    if (t > s && linked(lam[t - 1], lam[t], cut, ctol)) continue;  // not the first of its cluster
    if (t + 1 < s + m && linked(lam[t], lam[t + 1], cut, ctol)) continue;  // cluster: workgroup pass below
    if (rk[t] >= nvec) continue;
    gdouble* z = Z + t;  // element i at z[i * ld]
    if (fabs(lam[t]) <= cut || m == 1) {
      for (int i = 0; i < n; ++i) z[i * ld] = (m == 1 && fabs(lam[t]) > cut && i == s) ? 1.0 : 0.0;
      continue;
    }
    gdouble* u = scratch + t;  // slot t, interleaved with the other threads' slots
    gdouble* v = u + nn;
    gdouble* w = v + nn;
    gdouble* mult = w + nn;
    gdouble* piv = mult + nn;
    tri_factor(dd + s, ee + s, m, lam[t], fmax(tn * 1e-15, 1e-300), u, v, w, mult, piv, ld);
    for (int i = 0; i < n; ++i) z[i * ld] = (i >= s && i < s + m) ? start_value(i, t) : 0.0;
    // each solve takes the previous solution scaled to unit norm as its right-hand side
    double sc = 1.0;
    for (int it = 0; it < kInvIters; ++it) {
      const double q = tri_solve(m, u, v, w, mult, piv, z + s * ld, ld, sc);
      sc = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    }
    strided_scale(m, z + s * ld, ld, sc);
  }
  __syncthreads();
  // workgroup clusters: (first, last, block) listed in runs, members flagged in vsh
  for (int i = tid; i < n; i += bs) vsh[i] = 0.0;
  __syncthreads();
  if (tid == 0) {
    int nr = 0;
    for (int b = 0; b < nblk; ++b) {
      const int s = bstart[b], e = bstart[b + 1];
      int t = s;
      while (t < e) {
        int last = t;
        while (last + 1 < e && linked(lam[last], lam[last + 1], cut, ctol)) ++last;
        if (last > t && t >= t0 && t < t1) {
          runs[3 * nr] = t; runs[3 * nr + 1] = last; runs[3 * nr + 2] = b;
          // members flagged by their 1-based offset in the cluster (0: not wanted)
          for (int q = t; q <= last; ++q) vsh[q] = rk[q] < nvec ? double(q - t + 1) : 0.0;
          ++nr;
        }
        t = last + 1;
      }
    }
    sh_nruns = nr;
  }
  __syncthreads();
  const int nruns = sh_nruns;
  // simultaneous inverse iteration: every member solves with its own shift in parallel,
  // then each cluster is orthonormalised by the workgroup (classical Gram-Schmidt, twice)
  for (int it = 0; it < 3 && nruns > 0; ++it) {
    for (int p = tid; p < n; p += bs) {
      if (vsh[p] == 0.0) continue;
      int lo_b = 0, hi_b = nblk - 1;
      while (lo_b < hi_b) {
        const int mid = (lo_b + hi_b + 1) >> 1;
        if (bstart[mid] <= p) lo_b = mid; else hi_b = mid - 1;
      }
      const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
      gdouble* u = scratch + p;
      gdouble* v = u + nn;
      gdouble* w = v + nn;
      gdouble* mult = w + nn;
      gdouble* piv = mult + nn;
      gdouble* z = Z + p;
      if (it == 0) {
        // members' shifts spread by their offset in the cluster, as in the single-thread path
        tri_factor(dd + s, ee + s, m, lam[p] + (vsh[p] - 1.0) * 10.0 * 2.2e-16 * tn, fmax(tn * 1e-15, 1e-300), u, v,
                   w, mult, piv, ld);
        for (int i = 0; i < n; ++i) z[i * ld] = (i >= s && i < s + m) ? start_value(i, p) : 0.0;
      }
      // the workgroup normalises each member after its orthogonalisation below
      tri_solve(m, u, v, w, mult, piv, z + s * ld, ld, 1.0);
    }
    __syncthreads();
    for (int q = 0; q < nruns; ++q) {
      const int r0 = runs[3 * q], r1 = runs[3 * q + 1], b = runs[3 * q + 2];
      const int s = bstart[b], m = bstart[b + 1] - s;
      for (int j = r0; j <= r1; ++j) {
        if (vsh[j] == 0.0) continue;
        gdouble* z = Z + j;
        for (int pass = 0; pass < 2 && j > r0; ++pass) {
          for (int jj = r0 + wave; jj < j; jj += nw) {
            gcdouble* y = Z + jj;
            double dot = 0.0;
            if (vsh[jj] == 0.0) {
              if (lane == 0) psh[jj - r0] = 0.0;
              continue;
            }
            for (int i = s + lane; i < s + m; i += 64) dot += y[i * ld] * z[i * ld];
            dot = wave_sum_d(dot);
            if (lane == 0) psh[jj - r0] = dot;
          }
          __syncthreads();
          for (int i = s + tid; i < s + m; i += bs) {
            double acc = 0.0;
            for (int jj = r0; jj < j; ++jj)
              if (vsh[jj] != 0.0) acc += psh[jj - r0] * Z[i * ld + jj];
            z[i * ld] -= acc;
          }
          __syncthreads();
        }
        double part = 0.0;
        for (int i = s + tid; i < s + m; i += bs) part += z[i * ld] * z[i * ld];
        const double nn2 = block_sum(part, red, tid, bs);
        const double sc = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
        for (int i = s + tid; i < s + m; i += bs) z[i * ld] *= sc;
        __syncthreads();
      }
    }
  }
}

// 3b. The eigenvectors of T in descending order of their eigenvalues into the work area:
//     columns of rank below nvec, zero below the cut.  Each workgroup moves a tile of 32
//     positions x 64 rows through LDS (coalesced on both sides).
__global__ __launch_bounds__(256) void tridiag_sort_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double tile[32][65];
  __shared__ int rks[32];
  __shared__ int keep[32];
  const EigDesc D = descs[blockIdx.z];
  const int n = D.n;
  const int c0 = blockIdx.x * 32, i0 = blockIdx.y * 64;
  if (c0 >= n || i0 >= n) return;
  const int nvec = D.nvec < 0 ? n : min(D.nvec, n);
  if (nvec == 0) return;
  const int tid = threadIdx.x;
  const int64_t nn0 = (int64_t)n * n;
  gdouble* W = gbl(D.work);
  gcdouble* tail = tri_tail(W, n);
  const double shift = tail[3 * n], vcut = tail[5 * n + 1];
  gcdouble* glam = tail + 3 * n + 1;
  gcdouble* grank = glam + n;
  gcdouble* Z = gbl(D.V);  // element i of vector c at Z[i n + c]
  gdouble* ZT = W + 6 * nn0;
  if (tid < 32) {
    const int c = c0 + tid;
    rks[tid] = c < n ? int(grank[c]) : n;
    keep[tid] = c < n && fabs(glam[c] + shift) > vcut;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = tid + 256 * j, q = e & 31, r = e >> 5;
    const int i = i0 + r, c = c0 + q;
    tile[q][r] = (i < n && c < n) ? Z[(int64_t)i * n + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int e = tid + 256 * j, r = e & 63, q = e >> 6;
    const int i = i0 + r, c = c0 + q;
    if (i < n && c < n && rks[q] < nvec) ZT[i + (int64_t)rks[q] * n] = keep[q] ? tile[q][r] : 0.0;
  }
}

// 4. Back-transformation V = H_0 ... H_{n-3} Z_T: wavefront w of workgroup (x, p) owns
// columns 8x + 2w and 8x + 2w + 1 of problem p, lane l holds rows l + 64 j (j < ROWS).
// The reflectors go in pairs (k, k - 1): with a = v_k^T z, b = v_{k-1}^T z and
// c = v_{k-1}^T v_k from one round of wavefront sums,
//   H_{k-1} H_k z = z - d_k v_k - d_{k-1} v_{k-1},  d_k = beta_k a,
//   d_{k-1} = beta_{k-1} (b - c d_k),
// so a pair costs one chain of cross-lane sums instead of two.
template <int ROWS>
__global__ __launch_bounds__(256) void tridiag_back_kernel(const EigDesc* __restrict__ descs) {
  const EigDesc D = descs[blockIdx.y];
  const int n = D.n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = 8 * blockIdx.x + 2 * wave;
  if (c0 >= n || n > 64 * ROWS) return;
  gdouble* Vout = gbl(D.V);
  const int nvec = D.nvec < 0 ? n : min(D.nvec, n);
  if (c0 >= nvec) {  // columns beyond the wanted ones are zero
    for (int r = lane; r < n; r += 64) {
      Vout[r + (int64_t)c0 * n] = 0.0;
      if (c0 + 1 < n) Vout[r + (int64_t)(c0 + 1) * n] = 0.0;
    }
    return;
  }
  const bool two = c0 + 1 < nvec;
  const int64_t nn0 = (int64_t)n * n;
  gcdouble* A = gbl(D.work);
  gcdouble* ZT = A + 6 * nn0;
  gcdouble* betas = A + 7 * nn0;
  double z0[ROWS], z1[ROWS];
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int r = lane + 64 * j;
    z0[j] = r < n ? ZT[r + (int64_t)c0 * n] : 0.0;
    z1[j] = (r < n && two) ? ZT[r + (int64_t)(c0 + 1) * n] : 0.0;
  }
  // reflector k: v_r = A[r, k] for r > k (zero when beta_k = 0: the column then holds no
  // reflector)
  auto load = [&](int k, double beta, double (&v)[ROWS]) {
    gcdouble* vk = A + (int64_t)k * n;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const int r = lane + 64 * j;
      v[j] = (beta != 0.0 && r > k && r < n) ? vk[r] : 0.0;
    }
  };
  int k = n - 3;
  for (; k >= 1; k -= 2) {
    const double bk = betas[k], bl = betas[k - 1];
    double vk[ROWS], vl[ROWS];
    load(k, bk, vk);
    load(k - 1, bl, vl);
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, c = 0.0;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      a0 += vk[j] * z0[j];
      a1 += vk[j] * z1[j];
      b0 += vl[j] * z0[j];
      b1 += vl[j] * z1[j];
      c += vl[j] * vk[j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      b0 += __shfl_xor(b0, off, 64);
      b1 += __shfl_xor(b1, off, 64);
      c += __shfl_xor(c, off, 64);
    }
    const double dk0 = bk * a0, dk1 = bk * a1;
    const double dl0 = bl * (b0 - c * dk0), dl1 = bl * (b1 - c * dk1);
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      z0[j] -= dk0 * vk[j] + dl0 * vl[j];
      z1[j] -= dk1 * vk[j] + dl1 * vl[j];
    }
  }
  if (k == 0) {  // an odd number of reflectors: the last one alone
    const double bk = betas[0];
    double vk[ROWS];
    load(0, bk, vk);
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      a0 += vk[j] * z0[j];
      a1 += vk[j] * z1[j];
    }
    a0 = bk * wave_sum_d(a0);
    a1 = bk * wave_sum_d(a1);
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      z0[j] -= a0 * vk[j];
      z1[j] -= a1 * vk[j];
    }
  }
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int r = lane + 64 * j;
    if (r < n) {
      Vout[r + (int64_t)c0 * n] = z0[j];
      if (c0 + 1 < n) Vout[r + (int64_t)(c0 + 1) * n] = two ? z1[j] : 0.0;
    }
  }
}

static int tridiag_threads(int nmax) { return nmax <= 64 ? 256 : kTriThreads; }
static int panel_threads(int nmax) { return nmax <= 64 ? 256 : kPanelThreads; }

// LDS bytes: panel (3 + nw) n + 2 kTriPanel doubles; values 3 n doubles with n + 1 ints;
// vectors 7 n doubles with n + 1 + 3 (n/2 + 1) ints; ranks n doubles.
static size_t tridiag_panel_lds(int n, int threads) {
  return (size_t(3 + threads / 64) * n + 2 * kTriPanel) * sizeof(double);
}
static size_t tridiag_values_lds(int n) { return size_t(3) * n * sizeof(double) + size_t(n + 1) * sizeof(int); }
static size_t tridiag_vec_lds(int n) {
  return size_t(7) * n * sizeof(double) + size_t(n + 1 + 3 * (n / 2 + 1)) * sizeof(int);
}

// One-time kernel attribute set-up, shared by contexts that run in parallel host threads.
static std::mutex g_attr_mutex;

static void lds_opt_in(const void* fn, size_t shm, size_t* granted) {
  if (shm <= 65536) return;
  std::lock_guard<std::mutex> lock(g_attr_mutex);
  if (shm <= *granted) return;
  // the request is exactly the dynamic size: the kernel's static LDS counts against the
  // same per-workgroup limit, so asking for the device maximum can be refused
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)) == hipSuccess) *granted = shm;
  (void)hipGetLastError();
  if (shm > *granted) throw std::runtime_error("eig: tridiagonal solver needs more LDS than the device grants");
}

void launch_tri_prepare(const EigDesc* d, int nprob, int nmax, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  const int T = (nmax + kPrepTile - 1) / kPrepTile;
  hipLaunchKernelGGL(tridiag_copy_kernel, dim3(T * (T + 1) / 2, nprob), dim3(256), 0, s, d);
  PV_LAUNCH_CHECK();
  hipLaunchKernelGGL(tridiag_prepare_kernel, dim3(nprob), dim3(nmax <= 64 ? 256 : kRedThreads), 0, s, d);
  PV_LAUNCH_CHECK();
}

void launch_tri_panel(const EigDesc* d, int nprob, int nmax, int k0, hipStream_t s) {
  if (nprob <= 0 || k0 + 2 >= nmax) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  static size_t granted = 0;
  const int threads = panel_threads(nmax);
  const size_t shm = tridiag_panel_lds(nmax, threads);
  lds_opt_in((const void*)tridiag_panel_kernel, shm, &granted);
  hipLaunchKernelGGL(tridiag_panel_kernel, dim3(nprob), dim3(threads), shm, s, d, k0);
  PV_LAUNCH_CHECK();
}

void launch_tri_step(const EigDesc* d, int nprob, int nmax, int k, int G, hipStream_t s) {
  if (nprob <= 0 || k > std::max(nmax - 2, 0)) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  if (G < 1 || int64_t(nprob) * G > (int64_t(1) << 30)) throw std::runtime_error("eig: bad workgroup count");
  if (nmax <= 256)
    hipLaunchKernelGGL(tridiag_step_kernel<4>, dim3(nprob * G), dim3(kStepThreads), 0, s, d, k, G);
  else if (nmax <= 512)
    hipLaunchKernelGGL(tridiag_step_kernel<8>, dim3(nprob * G), dim3(kStepThreads), 0, s, d, k, G);
  else
    hipLaunchKernelGGL(tridiag_step_kernel<16>, dim3(nprob * G), dim3(kStepThreads), 0, s, d, k, G);
  PV_LAUNCH_CHECK();
}

// Attainable float64 MFMA rate of the device: each wavefront runs a chain of four
// independent 16x16x4 products per step on register operands only (no memory traffic)
// and writes its accumulators once.
__global__ __launch_bounds__(256) void mfma_rate_kernel(double* __restrict__ out, int iters) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = d4{0, 0, 0, 0};
  double a = 1e-3 * threadIdx.x, b = 1.0 + blockIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    a += 1e-30;
  }
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) t += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  gbl(out)[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

void launch_mfma_rate(double* out, int blocks, int iters, hipStream_t s) {
  if (blocks <= 0 || iters <= 0) return;
  hipLaunchKernelGGL(mfma_rate_kernel, dim3(blocks), dim3(256), 0, s, out, iters);
  PV_LAUNCH_CHECK();
}

void launch_tri_tail(const EigDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(tridiag_tail_kernel, dim3(nprob), dim3(kTailThreads), 0, s, d);
  PV_LAUNCH_CHECK();
}

int tri_tail_rows() { return kTailMax; }

void launch_tri_finish(const EigDesc* d, int nprob, hipStream_t s) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(tridiag_finish_kernel, dim3((nprob + 63) / 64), dim3(64), 0, s, d, nprob);
  PV_LAUNCH_CHECK();
}

void launch_eig_tridiag(const EigDesc* d, int nprob, int nmax, int phases, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  if (phases & 1) throw std::runtime_error("eig: the reduction runs through the panel launchers");
  const int threads = tridiag_threads(nmax);
  static size_t granted_values = 0, granted_vec = 0;
  const size_t shm_w = tridiag_values_lds(nmax), shm_v = tridiag_vec_lds(nmax);
  static size_t granted_values_wide = 0;
  lds_opt_in((const void*)tridiag_values_kernel<kSectLanes>, shm_w, &granted_values);
  lds_opt_in((const void*)tridiag_values_kernel<64>, shm_w, &granted_values_wide);
  lds_opt_in((const void*)tridiag_vec_kernel, shm_v, &granted_vec);
  if (phases & 2) {
    // one lane group per eigenvalue, several workgroups per matrix.  The Sturm sweeps are
    // bound by instruction issue in each wavefront; a small batch leaves most SIMDs idle,
    // so it takes a whole wavefront per eigenvalue (128 points per round, about half the
    // rounds of 16 points)
    if (int64_t(nprob) * nmax <= kSectWideMax) {
      const int pos = kValuesThreads / 64;
      const int parts = (nmax + pos - 1) / pos;
      hipLaunchKernelGGL(tridiag_values_kernel<64>, dim3(parts, nprob), dim3(kValuesThreads), shm_w, s, d);
    } else {
      const int parts = (nmax + kValuesPositions - 1) / kValuesPositions;
      hipLaunchKernelGGL(tridiag_values_kernel<kSectLanes>, dim3(parts, nprob), dim3(kValuesThreads), shm_w, s, d);
    }
    PV_LAUNCH_CHECK();
    hipLaunchKernelGGL(tridiag_rank_kernel, dim3(nprob), dim3(threads), size_t(nmax) * sizeof(double), s, d);
    PV_LAUNCH_CHECK();
  }
  if (phases & 4) {
    // the factor and solves of one vector stream through global memory: spread the
    // vectors of a matrix over several CUs
    const int parts = (nmax + kVectorPositions - 1) / kVectorPositions;
    hipLaunchKernelGGL(tridiag_vec_kernel, dim3(parts, nprob), dim3(kVectorPositions), shm_v, s, d);
    PV_LAUNCH_CHECK();
    hipLaunchKernelGGL(tridiag_sort_kernel, dim3((nmax + 31) / 32, (nmax + 63) / 64, nprob), dim3(256), 0, s, d);
    PV_LAUNCH_CHECK();
  }
  if (phases & 8) {
    const dim3 g((nmax + 7) / 8, nprob);
    if (nmax <= 256)
      hipLaunchKernelGGL(tridiag_back_kernel<4>, g, dim3(256), 0, s, d);
    else if (nmax <= 512)
      hipLaunchKernelGGL(tridiag_back_kernel<8>, g, dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL(tridiag_back_kernel<kBackRows>, g, dim3(256), 0, s, d);
    PV_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// Panel of the blocked Cholesky factorisation (one workgroup per matrix).  The first panel
// saves the original diagonal.  Wave 0 factors the kCholB x kCholB diagonal block in LDS
// (lanes along rows), dropping columns whose pivot is at most kCholDrop times their
// original diagonal entry; every thread then solves one row of the block below it,
// x L11^T = a, by forward substitution (dropped columns give zeros).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chol_panel_kernel(const CholDesc* __restrict__ descs, int j0) {
  __shared__ double L11[kCholB][kCholB + 1];
  __shared__ double dref[kCholB];
  const CholDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (j0 >= n) return;
  gdouble* A = gbl(D.A);
  const int lda = D.lda;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int jb = min(kCholB, n - j0);
  gdouble* dg = gbl(D.dg);
  if (j0 == 0) {
    for (int i = tid; i < n; i += bs) dg[i] = A[i + (int64_t)i * lda];
    __syncthreads();
  }
  for (int c = tid; c < jb; c += bs) dref[c] = dg[j0 + c];
  for (int e = tid; e < jb * jb; e += bs) {
    const int r = e % jb, c = e / jb;
    L11[r][c] = r >= c ? A[(j0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    for (int k = 0; k < jb; ++k) {
      const double d = L11[k][k];
      const double l = d > kCholDrop * dref[k] ? sqrt(d) : 0.0;
      const double inv = l > 0.0 ? 1.0 / l : 0.0;
      __builtin_amdgcn_wave_barrier();
      if (lane > k && lane < jb) L11[lane][k] *= inv;
      if (lane == 0) L11[k][k] = l;
      __builtin_amdgcn_wave_barrier();
      for (int c = k + 1; c < jb; ++c)
        if (lane >= c && lane < jb) L11[lane][c] -= L11[lane][k] * L11[c][k];
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  // the panel columns: zero above the diagonal, L11 on the diagonal block
  for (int e = tid; e < (j0 + jb) * jb; e += bs) {
    const int c = e / (j0 + jb), i = e - c * (j0 + jb);
    A[i + (int64_t)(j0 + c) * lda] = i < j0 + c ? 0.0 : L11[i - j0][c];
  }
  // rows below the diagonal block
  for (int i = j0 + jb + tid; i < n; i += bs) {
    double x[kCholB];
#pragma unroll
    for (int c = 0; c < kCholB; ++c) x[c] = c < jb ? A[i + (int64_t)(j0 + c) * lda] : 0.0;
#pragma unroll
    for (int c = 0; c < kCholB; ++c) {
      if (c >= jb) continue;
      double s = x[c];
#pragma unroll
      for (int k = 0; k < kCholB; ++k)
        if (k < c) s -= x[k] * L11[c][k];
      x[c] = L11[c][c] > 0.0 ? s / L11[c][c] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kCholB; ++c)
      if (c < jb) A[i + (int64_t)(j0 + c) * lda] = x[c];
  }
}

void launch_chol_panel(const CholDesc* d, int nprob, int j0, hipStream_t s) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(chol_panel_kernel, dim3(nprob), dim3(256), 0, s, d, j0);
  PV_LAUNCH_CHECK();
}

static size_t g_lds_limit = size_t(-1);

// Largest dynamic LDS accepted for the LDS-resident variants (0 when the opt-in fails).
static size_t eig_lds_limit() {
  std::lock_guard<std::mutex> lock(g_attr_mutex);
  if (g_lds_limit == size_t(-1)) {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
    (void)hipGetLastError();
    size_t want = v > 1024 ? size_t(v) - 1024 : 0;  // room for the static flag
    const void* fns[3] = {(const void*)jacobi_eig_kernel<0>, (const void*)jacobi_eig_kernel<1>,
                          (const void*)jacobi_eig_kernel<2>};
    for (const void* f : fns)
      if (want > 0 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) != hipSuccess) {
        (void)hipGetLastError();
        want = 0;
      }
    g_lds_limit = want;
  }
  return g_lds_limit;
}

int eig_mode(int n) {
  const size_t lim = eig_lds_limit();
  if (eig_lds_bytes(n, 2) <= lim) return 2;
  if (eig_lds_bytes(n, 1) <= lim) return 1;
  return 0;
}

void launch_eig(const EigDesc* d, int nprob, int nmax, int mode, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  const size_t shm = eig_lds_bytes(nmax, mode);
  if (shm > eig_lds_limit()) throw std::runtime_error("eig: LDS request above the device limit");
  const int threads = nmax <= 48 ? 256 : (nmax <= 96 ? 512 : 1024);
  if (mode == 2)
    hipLaunchKernelGGL(jacobi_eig_kernel<2>, dim3(nprob), dim3(threads), shm, s, d, 60);
  else if (mode == 1)
    hipLaunchKernelGGL(jacobi_eig_kernel<1>, dim3(nprob), dim3(threads), shm, s, d, 60);
  else
    hipLaunchKernelGGL(jacobi_eig_kernel<0>, dim3(nprob), dim3(threads), shm, s, d, 60);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// W-step: one workgroup per (output block, output state b').
// ---------------------------------------------------------------------------
// One workgroup per task: every thread owns kWElems elements of the task, computes their
// coordinates once and accumulates over the task's entries (read as uniform loads), so
// the kWElems gathers of an entry are issued together.  Tasks without entries write zeros.
__global__ __launch_bounds__(256) void wstep_kernel(const WTask* __restrict__ tasks,
                                                    const WEntry* __restrict__ entries) {
  const WTask t = tasks[blockIdx.x];
  const int rows = t.rows;
  int ar[kWElems], cr[kWElems];
  bool ok[kWElems];
  double acc[kWElems];
#pragma unroll
  for (int r = 0; r < kWElems; ++r) {
    const int x = t.x0 + r * 256 + (int)threadIdx.x;
    ok[r] = x < t.n;
    ar[r] = ok[r] ? x % rows : 0;
    cr[r] = ok[r] ? x / rows : 0;
    acc[r] = 0.0;
  }
  // entries four at a time with all their loads issued together; lanes past the end of the
  // block read element (0, 0) of the source and are not stored, so no load is guarded.  The
  // terms are added in entry order either way.
  int e = t.e0;
  for (; e + 4 <= t.e1; e += 4) {
    const WEntry E0 = entries[e], E1 = entries[e + 1], E2 = entries[e + 2], E3 = entries[e + 3];
    gcdouble* s0 = gbl(E0.src);
    gcdouble* s1 = gbl(E1.src);
    gcdouble* s2 = gbl(E2.src);
    gcdouble* s3 = gbl(E3.src);
    double x0[kWElems], x1[kWElems], x2[kWElems], x3[kWElems];
#pragma unroll
    for (int r = 0; r < kWElems; ++r) {
      x0[r] = s0[ar[r] + E0.ld * cr[r]];
      x1[r] = s1[ar[r] + E1.ld * cr[r]];
      x2[r] = s2[ar[r] + E2.ld * cr[r]];
      x3[r] = s3[ar[r] + E3.ld * cr[r]];
    }
#pragma unroll
    for (int r = 0; r < kWElems; ++r) {
      acc[r] += E0.val * x0[r];
      acc[r] += E1.val * x1[r];
      acc[r] += E2.val * x2[r];
      acc[r] += E3.val * x3[r];
    }
  }
  for (; e < t.e1; ++e) {
    const WEntry E = entries[e];
    gcdouble* src = gbl(E.src);
#pragma unroll
    for (int r = 0; r < kWElems; ++r) acc[r] += E.val * src[ar[r] + E.ld * cr[r]];
  }
  gdouble* out = gbl(t.out);
#pragma unroll
  for (int r = 0; r < kWElems; ++r)
    if (ok[r]) out[ar[r] + t.ldo * cr[r]] = acc[r];
}

void launch_wstep(const WTask* tasks, int ntasks, const WEntry* entries, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(wstep_kernel, dim3(ntasks), dim3(256), 0, s, tasks, entries);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched block copy with scale, and column scaling.
// ---------------------------------------------------------------------------
__global__ void copy_kernel(const CopyDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const CopyDesc c = d[lo];
  const int64_t x = e - c.elem0;
  const int i = int(x % c.rows), j = int(x / c.rows);
  c.dst[i + (int64_t)j * c.ldd] = c.src ? c.alpha * c.src[i + (int64_t)j * c.lds] : c.alpha;
}

void launch_copy(const CopyDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

__global__ void scale_kernel(const ScaleDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const ScaleDesc c = d[lo];
  const int64_t x = e - c.elem0;
  const int i = int(x % c.rows), j = int(x / c.rows);
  double f = c.s[j];
  if (c.sqrt_s) f = sqrt(fmax(f, 0.0));
  if (c.invert) f = f != 0.0 ? 1.0 / f : 0.0;
  c.dst[i + (int64_t)j * c.ldd] = f * c.src[i + (int64_t)j * c.lds];
}

void launch_scale(const ScaleDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Sum of squares with wavefront shuffles: per-lane partial sums, a 64-lane
// butterfly (__shfl_xor), one value per wave through LDS, and a fixed-order final sum
// by a single workgroup, so the result is bitwise reproducible.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(1024) void sumsq_kernel(const double* __restrict__ x, int64_t n, double* out) {
  __shared__ double part[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += x[i] * x[i];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += part[w];
    *out = t;
  }
}

void launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
  PV_LAUNCH_CHECK();
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = v;
}

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n, v);
  PV_LAUNCH_CHECK();
}

}  // namespace pv
