// Device kernels of the CCSD derivative-coupling library (gfx950 / CDNA4).
//
// * gemm_f64      : batched C = alpha op(A) op(B) + beta C on the FP64 matrix
//                   cores (v_mfma_f64_16x16x4f64), LDS-staged 64x64x16 tiles,
//                   four 64-wide waves per workgroup, each owning a 32x32 block.
// * view_gather / view_scatter : one generic strided data-movement kernel
//                   pair; every permutation, block extraction, symmetrisation
//                   and axpy of the contraction engine is one of these.
// * reductions    : deterministic two-pass dot products and max-abs.
// * elementwise   : orbital-energy denominators (Jacobi / Davidson
//                   preconditioners), packed-metric weights.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cmath>

#include "kernels.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// Output row of accumulator element v for lane group lk (= lane / 16) of the
// fp32 16x16x4 MFMA (measured: 4 lk + v; the fp64 16x16x4 MFMA uses lk + 4 v).
#define F32_ROW(lk, v) (4 * (lk) + (v))

namespace nm {

// --------------------------------------------------------------------- GEMM
// Tile: BM x BN x BK = 64 x 64 x 16, 256 threads = 4 waves arranged 2 x 2.
// LDS holds A as As[k][m] and B as Bs[k][n] so that the MFMA operand of lane
// l (row/col l % 16, k = l / 16) is read from consecutive addresses.
constexpr int BM = 64, BN = 64, BK = 16, PAD = 1;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, int64_t lda,
    int64_t sA, const double* __restrict__ B, int64_t ldb, int64_t sB, double beta,
    double* __restrict__ C, int64_t ldc, int64_t sC, int Klast) {
  __shared__ double As[BK][BM + PAD];
  __shared__ double Bs[BK][BN + PAD];
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (Klast > 0 && blockIdx.z == gridDim.z - 1) K = Klast;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int m, k;
      if (!TA) { m = e >> 4; k = e & 15; } else { k = e >> 6; m = e & 63; }
      const int gm = m0 + m, gk = k0 + k;
      double val = 0.0;
      if (gm < M && gk < K) val = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[k][m] = val;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int k, n;
      if (!TB) { k = e >> 6; n = e & 63; } else { n = e >> 4; k = e & 15; }
      const int gn = n0 + n, gk = k0 + k;
      double val = 0.0;
      if (gn < N && gk < K) val = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[k][n] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of v_mfma_f64_16x16x4f64: lane l, element v -> row l/16 + 4 v, col l % 16.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * 32 + i * 16 + lk + 4 * v;
        const int gn = n0 + wn * 32 + j * 16 + lr;
        if (gm < M && gn < N) {
          double* c = C + (int64_t)gm * ldc + gn;
          const double r = alpha * acc[i][j][v];
          *c = (beta == 0.0) ? r : r + beta * (*c);
        }
      }
}

// Large-tile variant: 128 x 128 x 16 per workgroup of 8 waves (4 x 2), each
// wave a 32 x 64 block (2 x 4 MFMA tiles, 32 fp64 accumulators per lane), so
// that two workgroups (four waves per SIMD) share a CU and hide each other's
// global-load latency.  The next K tile is
// prefetched into registers while the current one is consumed from LDS
// (double-buffered), so one barrier per K tile suffices.
//
// LDS layouts follow the global layout of each operand so that both the
// stores and the MFMA operand reads are free of bank conflicts:
//  * an operand whose K index is contiguous in memory (A row-major, B
//    transposed) is kept as [row][k] with a row stride of 17 doubles (34
//    banks): the 16 lanes of an MFMA operand read hit 16 distinct bank pairs;
//  * an operand whose M/N index is contiguous (A transposed, B row-major) is
//    kept as [k][row] with a row stride of 144 doubles (a 32-bank shift
//    between successive k rows, so the two half-waves read disjoint banks).
// Tiles are ordered so that the M tiles sharing one B column tile run back to
// back on the same XCD (workgroups are dealt round-robin over the 8 XCDs).
// Workgroups are dealt round-robin over the 8 XCDs (workgroup b runs on XCD
// b % 8).  XCD x is given a contiguous range of tile indices (a bijection on
// [0, total) for any total), so that tiles sharing operand panels run on the
// same XCD at the same time and meet in its L2.
__device__ inline int xcd_tile(int b, int total) {
  const int per = total >> 3, rem = total & 7;
  const int x = b & 7, s = b >> 3;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + s;
}

constexpr int LBM = 128, LBN = 128, LBK = 16;
constexpr int LKS = LBK + 1;     // [row][k] stride
constexpr int LRS = 128 + 16;    // [k][row] stride

template <bool TA, bool TB, int NT>
__global__ __launch_bounds__(NT, 4) void gemm_f64_big_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, int64_t lda,
    int64_t sA, const double* __restrict__ B, int64_t ldb, int64_t sB, double beta,
    double* __restrict__ C, int64_t ldc, int64_t sC, int Klast) {
  // NT = 256: 4 waves (2 x 2), each 64 x 64 (4 x 4 MFMA tiles), 1 wave/SIMD.
  // NT = 512: 8 waves (4 x 2), each 32 x 64 (2 x 4 MFMA tiles), 2 waves/SIMD.
  constexpr int WM = (NT == 256) ? 2 : 4;          // waves along M
  constexpr int TR = LBM / WM;                      // rows per wave
  constexpr int FI = TR / 16;                       // MFMA row tiles per wave
  constexpr int PER = (LBM * LBK) / NT;             // elements per thread per operand
  constexpr int RSTEP = NT / 16;                    // row step of the K-contiguous pattern
  constexpr int KSTEP = NT / 128;                   // k step of the row-contiguous pattern
  constexpr int ASZ = TA ? LBK * LRS : LBM * LKS;
  constexpr int BSZ = TB ? LBN * LKS : LBK * LRS;
  __shared__ double As[2][ASZ];
  __shared__ double Bs[2][BSZ];
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  if (Klast > 0 && blockIdx.z == gridDim.z - 1) K = Klast;
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy;
  int bid = blockIdx.x + gx * blockIdx.y;
  bid = xcd_tile(bid, total);
  const int tm = bid % gy, tn = bid / gy;
  const int m0 = tm * LBM, n0 = tn * LBN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // Per-thread load pattern (PER elements of each operand per K tile):
  //  K-contiguous operand : row = (tid >> 4) + RSTEP r, k = tid & 15
  //  row-contiguous operand: k = (tid >> 7) + KSTEP r,  row = tid & 127
  const int a_row0 = TA ? (tid & 127) : (tid >> 4);
  const int a_k0 = TA ? (tid >> 7) : (tid & 15);
  const int b_row0 = TB ? (tid >> 4) : (tid & 127);
  const int b_k0 = TB ? (tid & 15) : (tid >> 7);
  const double* pa = TA ? A + (int64_t)a_k0 * lda + (m0 + a_row0) : A + (int64_t)(m0 + a_row0) * lda + a_k0;
  const double* pb = TB ? B + (int64_t)(n0 + b_row0) * ldb + b_k0 : B + (int64_t)b_k0 * ldb + (n0 + b_row0);
  const int64_t a_rstep = TA ? KSTEP * lda : RSTEP * lda;
  const int64_t b_rstep = TB ? RSTEP * ldb : KSTEP * ldb;
  const int64_t a_kstep = TA ? (int64_t)LBK * lda : LBK;
  const int64_t b_kstep = TB ? LBK : (int64_t)LBK * ldb;

  v4d acc[FI][4];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  double ra[PER], rb[PER];
  auto gload = [&](int t) {
    const int kb = t * LBK;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int row = TA ? a_row0 : a_row0 + RSTEP * r;
      const int k = TA ? a_k0 + KSTEP * r : a_k0;
      const bool ok = (m0 + row < M) && (kb + k < K);
      ra[r] = ok ? pa[t * a_kstep + r * a_rstep] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int row = TB ? b_row0 + RSTEP * r : b_row0;
      const int k = TB ? b_k0 : b_k0 + KSTEP * r;
      const bool ok = (n0 + row < N) && (kb + k < K);
      rb[r] = ok ? pb[t * b_kstep + r * b_rstep] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (TA) As[buf][(a_k0 + KSTEP * r) * LRS + a_row0] = ra[r];
      else As[buf][(a_row0 + RSTEP * r) * LKS + a_k0] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (TB) Bs[buf][(b_row0 + RSTEP * r) * LKS + b_k0] = rb[r];
      else Bs[buf][(b_k0 + KSTEP * r) * LRS + b_row0] = rb[r];
    }
  };
  const int nk = (K + LBK - 1) / LBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) gload(t + 1);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < LBK; kk += 4) {
      double a[FI], bb[4];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        const int row = wm * TR + i * 16 + lr, k = kk + lk;
        a[i] = TA ? as[k * LRS + row] : as[row * LKS + k];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wn * 64 + j * 16 + lr, k = kk + lk;
        bb[j] = TB ? bs[row * LKS + k] : bs[k * LRS + row];
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * TR + i * 16 + lk + 4 * v;
        const int gn = n0 + wn * 64 + j * 16 + lr;
        if (gm < M && gn < N) {
          double* c = C + (int64_t)gm * ldc + gn;
          const double r = alpha * acc[i][j][v];
          *c = (beta == 0.0) ? r : r + beta * (*c);
        }
      }
}


// FP32 variant of the large-tile kernel for the mixed-precision path: fp32
// operands (packed by the caller), v_mfma_f32_16x16x4f32 with fp32
// accumulation, fp64 epilogue C = alpha * acc + beta * C.  Same 128 x 128
// tiling and XCD-grouped tile order as the fp64 kernel, with a K step of 32
// (half the barriers per MFMA of a 16 step; two workgroups of 74 KB LDS fit a
// CU).  LDS strides: [row][k] 34 floats (2 mod 32: the 16 rows x 2 k of a
// half-wave's operand read hit 32 distinct banks), [k][row] 144 floats
// (16 mod 32: 2 k x 16 rows again distinct).
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int FBK = 32, FKS = FBK + 2, FRS = 128 + 16;

template <bool TA, bool TB>
__global__ __launch_bounds__(512, 4) void gemm_f32acc_big_kernel(
    int M, int N, int K, double alpha, const float* __restrict__ A, int64_t lda, int64_t sA,
    const float* __restrict__ B, int64_t ldb, int64_t sB, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sC, int Klast) {
  constexpr int NT = 512, WM = 4, TR = LBM / WM, FI = TR / 16;
  constexpr int PER = (LBM * FBK) / NT, RSTEP = NT / FBK, KSTEP = NT / 128;
  constexpr int ASZ = TA ? FBK * FRS : LBM * FKS;
  constexpr int BSZ = TB ? LBN * FKS : FBK * FRS;
  __shared__ float As[2][ASZ];
  __shared__ float Bs[2][BSZ];
  // grid.z: batch entries, or K chunks of a split-K product (the last chunk
  // Klast long when Klast > 0)
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  if (Klast > 0 && blockIdx.z == gridDim.z - 1) K = Klast;
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy;
  int bid = blockIdx.x + gx * blockIdx.y;
  bid = xcd_tile(bid, total);
  const int tm = bid % gy, tn = bid / gy;
  const int m0 = tm * LBM, n0 = tn * LBN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int a_row0 = TA ? (tid & 127) : (tid / FBK);
  const int a_k0 = TA ? (tid >> 7) : (tid % FBK);
  const int b_row0 = TB ? (tid / FBK) : (tid & 127);
  const int b_k0 = TB ? (tid % FBK) : (tid >> 7);
  const float* pa = TA ? A + (int64_t)a_k0 * lda + (m0 + a_row0) : A + (int64_t)(m0 + a_row0) * lda + a_k0;
  const float* pb = TB ? B + (int64_t)(n0 + b_row0) * ldb + b_k0 : B + (int64_t)b_k0 * ldb + (n0 + b_row0);
  const int64_t a_rstep = TA ? KSTEP * lda : RSTEP * lda;
  const int64_t b_rstep = TB ? RSTEP * ldb : KSTEP * ldb;
  const int64_t a_kstep = TA ? (int64_t)FBK * lda : FBK;
  const int64_t b_kstep = TB ? FBK : (int64_t)FBK * ldb;
  v4f acc[FI][4];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  float ra[PER], rb[PER];
  auto gload = [&](int t) {
    const int kb = t * FBK;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int row = TA ? a_row0 : a_row0 + RSTEP * r;
      const int k = TA ? a_k0 + KSTEP * r : a_k0;
      const bool ok = (m0 + row < M) && (kb + k < K);
      ra[r] = ok ? pa[t * a_kstep + r * a_rstep] : 0.f;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int row = TB ? b_row0 + RSTEP * r : b_row0;
      const int k = TB ? b_k0 : b_k0 + KSTEP * r;
      const bool ok = (n0 + row < N) && (kb + k < K);
      rb[r] = ok ? pb[t * b_kstep + r * b_rstep] : 0.f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (TA) As[buf][(a_k0 + KSTEP * r) * FRS + a_row0] = ra[r];
      else As[buf][(a_row0 + RSTEP * r) * FKS + a_k0] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (TB) Bs[buf][(b_row0 + RSTEP * r) * FKS + b_k0] = rb[r];
      else Bs[buf][(b_k0 + KSTEP * r) * FRS + b_row0] = rb[r];
    }
  };
  const int nk = (K + FBK - 1) / FBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) gload(t + 1);
    const float* as = As[cur];
    const float* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < FBK; kk += 4) {
      float a[FI], bb[4];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        const int row = wm * TR + i * 16 + lr, k = kk + lk;
        a[i] = TA ? as[k * FRS + row] : as[row * FKS + k];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wn * 64 + j * 16 + lr, k = kk + lk;
        bb[j] = TB ? bs[row * FKS + k] : bs[k * FRS + row];
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * TR + i * 16 + F32_ROW(lk, v);
        const int gn = n0 + wn * 64 + j * 16 + lr;
        if (gm < M && gn < N) {
          double* c = C + (int64_t)gm * ldc + gn;
          const double r = alpha * (double)acc[i][j][v];
          *c = (beta == 0.0) ? r : r + beta * (*c);
        }
      }
}

int gemm_f32acc(hipStream_t s, bool ta, bool tb, int M, int N, int K, int batch, double alpha,
                const float* A, int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB,
                double beta, double* C, int64_t ldc, int64_t sC, int Klast) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  if (K <= 0) return -1;
  if (batch > 32768) {   // grid.z limit: launch in chunks
    for (int b0 = 0; b0 < batch; b0 += 32768) {
      const int nb = batch - b0 < 32768 ? batch - b0 : 32768;
      int rc = gemm_f32acc(s, ta, tb, M, N, K, nb, alpha, A + (int64_t)b0 * sA, lda, sA,
                           B + (int64_t)b0 * sB, ldb, sB, beta, C + (int64_t)b0 * sC, ldc, sC,
                           b0 + nb == batch ? Klast : 0);
      if (rc) return rc;
    }
    return 0;
  }
  dim3 grid((N + LBN - 1) / LBN, (M + LBM - 1) / LBM, batch);
#define NM_F32(TA_, TB_) \
  hipLaunchKernelGGL((gemm_f32acc_big_kernel<TA_, TB_>), grid, dim3(512), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast)
  if (!ta && !tb) NM_F32(false, false);
  else if (!ta && tb) NM_F32(false, true);
  else if (ta && !tb) NM_F32(true, false);
  else NM_F32(true, true);
#undef NM_F32
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ------------------------------------------------- BF16 split-precision GEMM
// C[m][n] = alpha * sum_k A[m][k] B[k][n] + beta * C with each fp32 operand
// carried as a bfloat16 pair x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
// so that x is held to about 2^-16 relative; every product is formed as
// al*bh + ah*bl + ah*bh (the lo*lo term, ~2^-16 of the product, is dropped) on
// the bf16 matrix cores (v_mfma_f32_16x16x32_bf16) with fp32 accumulation and
// an fp64 epilogue.  Operands are K-contiguous pair arrays, A [M][2 Kp] and
// B^T [N][2 Kp] (uint16 storage of bf16), hi and lo interleaved in 16-byte
// chunks: element k of a row has its hi at 2 (k - k % 8) + k % 8 and its lo 8
// further, so that a K step of 32 reads 128 contiguous bytes of a row (a whole
// cache line; separate hi and lo rows would use half of two lines each, and
// the launches ran 18 % longer).  Leading dimensions lda / ldb (uint16 units,
// >= 2 K) multiples of 8, K zero-padded to a multiple of 32, so that every
// global load and LDS access is a 16-byte vector and needs no K bound; K
// offset k0 of a split sits 2 k0 along the row.  MFMA lane layout (checked on the
// device): lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// for j < 8 and receives D rows 4 (l / 16) + v, column l % 16.
// Tiles 128 x 128 x 32, 512 threads = 8 waves of 32 x 64 outputs, double-
// buffered LDS rows of 32 bf16 with the 16-byte chunks XOR-swizzled (64 KB, two
// workgroups per CU), XCD-grouped tile order as the other kernels.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// 16-byte register chunk (a native vector: a HIP uint4 is a struct that is
// copied by memcpy and can be left in private or shared memory)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int HBK = 32, HKS = 32;
// 16-byte chunk c of tile row r sits at chunk c ^ ((r >> 1) & 3).  An operand
// read has lane l take chunk l / 16 of row l % 16 (16 bytes a lane, ds_read_b128);
// with this permutation it runs at the rate of a contiguous 1 KB read, where
// c ^ ((r >> 2) & 3) or no swizzle take twice the LDS cycles (bank conflicts,
// measured).  The staging stores write 16 whole rows a wave either way.
__device__ inline int swz(int r, int c) { return r * HKS + 8 * (c ^ ((r >> 1) & 3)); }

__global__ __launch_bounds__(512, 2) void gemm_bf16x3_kernel(
    int M, int N, int K, double alpha, const uint16_t* __restrict__ A, int64_t lda, int64_t sA,
    const uint16_t* __restrict__ B, int64_t ldb, int64_t sB, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sC, int Klast) {
  __shared__ __attribute__((aligned(16))) uint16_t S[2][4][128 * HKS];
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  if (Klast > 0 && blockIdx.z == gridDim.z - 1) K = Klast;
  const int gx = gridDim.x, gy = gridDim.y;
  int bid = blockIdx.x + gx * blockIdx.y;
  bid = xcd_tile(bid, gx * gy);
  const int tm = bid % gy, tn = bid / gy;
  const int m0 = tm * 128, n0 = tn * 128;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lr = lane & 15, lk = lane >> 4;
  // global loads: row tid / 4 of the tile, the hi and lo chunks of the 8
  // consecutive k at 8 (tid % 4)
  const int grow = tid >> 2, gch = (tid & 3) * 8;
  const bool aok = m0 + grow < M, bok = n0 + grow < N;
  const int64_t aoff = (int64_t)(aok ? m0 + grow : 0) * lda + 2 * gch;
  const int64_t boff = (int64_t)(bok ? n0 + grow : 0) * ldb + 2 * gch;
  const uint4 zero = {0u, 0u, 0u, 0u};
  uint4 r0, r1, r2, r3;
  auto gload = [&](int t) {
    const int64_t k0 = 2 * (int64_t)t * HBK;
    r0 = aok ? *(const uint4*)(A + aoff + k0) : zero;
    r1 = aok ? *(const uint4*)(A + aoff + k0 + 8) : zero;
    r2 = bok ? *(const uint4*)(B + boff + k0) : zero;
    r3 = bok ? *(const uint4*)(B + boff + k0 + 8) : zero;
  };
  auto sstore = [&](int buf) {
    const int o = swz(grow, gch >> 3);
    *(uint4*)&S[buf][0][o] = r0;
    *(uint4*)&S[buf][1][o] = r1;
    *(uint4*)&S[buf][2][o] = r2;
    *(uint4*)&S[buf][3][o] = r3;
  };
  v4f acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nk = K / HBK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) gload(t + 1);
    bf16x8 ah[2], al[2], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int o = swz(wm * 32 + i * 16 + lr, lk);
      ah[i] = *(const bf16x8*)&S[cur][0][o];
      al[i] = *(const bf16x8*)&S[cur][1][o];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = swz(wn * 64 + j * 16 + lr, lk);
      bh[j] = *(const bf16x8*)&S[cur][2][o];
      bl[j] = *(const bf16x8*)&S[cur][3][o];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    if (t + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * 32 + i * 16 + 4 * lk + v;
        const int gn = n0 + wn * 64 + j * 16 + lr;
        if (gm < M && gn < N) {
          double* c = C + (int64_t)gm * ldc + gn;
          const double r = alpha * (double)acc[i][j][v];
          *c = (beta == 0.0) ? r : r + beta * (*c);
        }
      }
}

// Large-tile variant for one workgroup per CU: BM x BN x 32 tiles (256 x 256
// or 256 x 128) over 8 waves of WM x WN, each wave a (BM / WM) x (BN / WN)
// block of FI x FJ MFMA tiles, so that every fragment read from LDS feeds FJ
// (A) or FI (B) products and a tile's operand panels are fetched once per
// BM x BN outputs (a quarter of the 128 x 128 kernel's panel traffic).  LDS:
// two stages of the four 32-wide bf16 row arrays (A hi, A lo, B hi, B lo),
// 256 (BM + BN) bytes in all (128 KB at 256 x 256), with the same XOR-swizzled
// 16-byte chunks as the 128 x 128 kernel.  Each thread moves
// (BM + BN) / 64 16-byte chunks per K step through registers, eight lanes
// to a row's 128-byte line (measured 3 % faster than four lanes to each of
// its hi and lo halves: a load instruction then touches half as many
// lines).  PD = 1: the next K step is loaded while this one is multiplied;
// PD = 2 (two register
// sets, the loop unrolled by two so that each set has fixed registers): the
// K step after next, so a global load has two steps of products to arrive.
// PD = 3: the fragments of the next K step are read from LDS into a second
// register set while this step's products run (and the next-but-one step's
// chunks are stored), so no product waits for an LDS read after the barrier.
// Every load is unconditional (past the last step the last one is read
// again), which keeps the waits at the LDS stores fixed.  The three products
// of a fragment pair are issued one per row block and then over the column
// blocks (FJ independent accumulators between dependent MFMAs).
template <int BM, int BN, int WM, int WN, int PD>
__global__ __launch_bounds__(WM * WN * 64, 1) void gemm_bf16x3_big_kernel(
    int M, int N, int K, double alpha, const uint16_t* __restrict__ A, int64_t lda, int64_t sA,
    const uint16_t* __restrict__ B, int64_t ldb, int64_t sB, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sC, int Klast) {
  static_assert(WM * WN == 8, "eight waves");
  static_assert(PD == 1 || PD == 2 || PD == 3, "pipeline variant");
  constexpr int TM = BM / WM, TN = BN / WN, FI = TM / 16, FJ = TN / 16;
  // 16-byte chunks per thread and operand per K step: rows / RP, with
  // RP = threads / 8 rows staged per pass (a row's K step is 8 chunks: hi and
  // lo of four groups of 8 k, one whole 128-byte line)
  constexpr int RP = WM * WN * 8, RA = BM / RP, RB = BN / RP;
  __shared__ __attribute__((aligned(16))) uint16_t SA[2][2][BM * HKS];
  __shared__ __attribute__((aligned(16))) uint16_t SB[2][2][BN * HKS];
  const int64_t bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  if (Klast > 0 && blockIdx.z == gridDim.z - 1) K = Klast;
  const int gx = gridDim.x, gy = gridDim.y;
  int bid = blockIdx.x + gx * blockIdx.y;
  bid = xcd_tile(bid, gx * gy);
  const int tm = bid % gy, tn = bid / gy;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int lr = lane & 15, lk = lane >> 4;
  // this thread's rows: (tid >> 3) + RP r, chunk tid & 7 of the row's K
  // step (the hi, for even chunks, or the lo half of k group (tid & 7) / 2),
  // of A (r < RA) and B (r < RB): eight lanes read a row's whole line
  const int row0 = tid >> 3, ch = tid & 7;
  int64_t aoff[RA], boff[RB];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const bool ok = m0 + row0 + RP * r < M;
    aoff[r] = (int64_t)(ok ? m0 + row0 + RP * r : 0) * lda + 8 * ch;
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const bool ok = n0 + row0 + RP * r < N;
    boff[r] = (int64_t)(ok ? n0 + row0 + RP * r : 0) * ldb + 8 * ch;
  }
  // rows outside the matrix read row 0 of the panel instead (always valid):
  // they only reach accumulators of output rows or columns that are never
  // stored, so they need no zeroing
  u32x4 ra0[RA], rb0[RB];
  u32x4 ra1[RA], rb1[RB];
  v4f acc[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int nk = K / HBK;
  // offset of K step t along a pair row (clamped to the last step)
#define NM_KOFF(t) ((int64_t)((t) < nk ? (t) : nk - 1) * (2 * HBK))
#define NM_LOAD(S, KO)                                                       \
  _Pragma("unroll") for (int r = 0; r < RA; ++r) ra##S[r] =                  \
      *(const u32x4*)(A + aoff[r] + (KO));                                   \
  _Pragma("unroll") for (int r = 0; r < RB; ++r) rb##S[r] =                  \
      *(const u32x4*)(B + boff[r] + (KO));
#define NM_STORE(S, G)                                                       \
  _Pragma("unroll") for (int r = 0; r < RA; ++r)                             \
      *(u32x4*)&SA[G][ch & 1][swz(row0 + RP * r, ch >> 1)] = ra##S[r];       \
  _Pragma("unroll") for (int r = 0; r < RB; ++r)                             \
      *(u32x4*)&SB[G][ch & 1][swz(row0 + RP * r, ch >> 1)] = rb##S[r];
#define NM_COMPUTE(G)                                                                             \
  {                                                                                               \
    bf16x8 fbh[FJ], fbl[FJ];                                                                      \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                              \
      const int o = swz(wn * TN + j * 16 + lr, lk);                                               \
      fbh[j] = *(const bf16x8*)&SB[G][0][o];                                                      \
      fbl[j] = *(const bf16x8*)&SB[G][1][o];                                                      \
    }                                                                                             \
    _Pragma("unroll") for (int i = 0; i < FI; ++i) {                                              \
      const int o = swz(wm * TM + i * 16 + lr, lk);                                               \
      const bf16x8 fah = *(const bf16x8*)&SA[G][0][o];                                            \
      const bf16x8 fal = *(const bf16x8*)&SA[G][1][o];                                            \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                  \
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal, fbh[j], acc[i][j], 0, 0, 0);               \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                  \
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah, fbl[j], acc[i][j], 0, 0, 0);               \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                  \
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah, fbh[j], acc[i][j], 0, 0, 0);               \
    }                                                                                             \
  }
#define NM_FRAGS(S, G)                                                                            \
  _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                                \
    const int o = swz(wn * TN + j * 16 + lr, lk);                                                 \
    qbh##S[j] = *(const bf16x8*)&SB[G][0][o];                                                     \
    qbl##S[j] = *(const bf16x8*)&SB[G][1][o];                                                     \
  }                                                                                               \
  _Pragma("unroll") for (int i = 0; i < FI; ++i) {                                                \
    const int o = swz(wm * TM + i * 16 + lr, lk);                                                 \
    qah##S[i] = *(const bf16x8*)&SA[G][0][o];                                                     \
    qal##S[i] = *(const bf16x8*)&SA[G][1][o];                                                     \
  }
#define NM_MMA(S)                                                                                 \
  _Pragma("unroll") for (int i = 0; i < FI; ++i) {                                                \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                    \
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(qal##S[i], qbh##S[j], acc[i][j], 0, 0, 0);        \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                    \
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(qah##S[i], qbl##S[j], acc[i][j], 0, 0, 0);        \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) acc[i][j] =                                    \
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(qah##S[i], qbh##S[j], acc[i][j], 0, 0, 0);        \
  }
  // (the scheduling barriers keep each step's loads ahead of its products and
  // its LDS stores, which wait for older loads, behind them)
  NM_LOAD(0, 0)
  NM_STORE(0, 0)
  if constexpr (PD == 3) {
    // fragment register sets; stage s of LDS holds step s mod 2 ahead
    bf16x8 qah0[FI], qal0[FI], qbh0[FJ], qbl0[FJ];
    bf16x8 qah1[FI], qal1[FI], qbh1[FJ], qbl1[FJ];
    NM_LOAD(0, NM_KOFF(1))
    __syncthreads();
    NM_FRAGS(0, 0)
    NM_STORE(0, 1)
    NM_LOAD(0, NM_KOFF(2))
    __syncthreads();
    int t = 0;
    for (; t + 1 < nk; t += 2) {
      // set 0: fragments of step t; stage 1: step t + 1; registers: step t + 2
      asm volatile("" ::: "memory");
      NM_FRAGS(1, 1)
      __builtin_amdgcn_sched_barrier(0);
      NM_MMA(0)
      __builtin_amdgcn_sched_barrier(0);
      NM_STORE(0, 0)
      NM_LOAD(0, NM_KOFF(t + 3))
      __syncthreads();
      asm volatile("" ::: "memory");
      // set 1: step t + 1; stage 0: step t + 2; registers: step t + 3
      NM_FRAGS(0, 0)
      __builtin_amdgcn_sched_barrier(0);
      NM_MMA(1)
      __builtin_amdgcn_sched_barrier(0);
      NM_STORE(0, 1)
      NM_LOAD(0, NM_KOFF(t + 4))
      __syncthreads();
    }
    if (t < nk) {   // odd step count: the last step's fragments are in set 0
      NM_MMA(0)
    }
  } else if constexpr (PD == 1) {
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
      const int cur = t & 1;
      NM_LOAD(0, NM_KOFF(t + 1))
      __builtin_amdgcn_sched_barrier(0);
      NM_COMPUTE(cur)
      __builtin_amdgcn_sched_barrier(0);
      NM_STORE(0, cur ^ 1)
      __syncthreads();
    }
  } else {
    // (the empty asm statements with a memory clobber keep the compiler's
    // loop transformations from moving loads between the two halves)
    NM_LOAD(1, NM_KOFF(1))
    __syncthreads();
    int t = 0;
    for (; t + 1 < nk; t += 2) {
      // stage 0 holds step t, set 1 step t + 1 (in flight)
      asm volatile("" ::: "memory");
      NM_LOAD(0, NM_KOFF(t + 2))
      __builtin_amdgcn_sched_barrier(0);
      NM_COMPUTE(0)
      __builtin_amdgcn_sched_barrier(0);
      NM_STORE(1, 1)
      __syncthreads();
      asm volatile("" ::: "memory");
      // stage 1 holds step t + 1, set 0 step t + 2 (in flight)
      NM_LOAD(1, NM_KOFF(t + 3))
      __builtin_amdgcn_sched_barrier(0);
      NM_COMPUTE(1)
      __builtin_amdgcn_sched_barrier(0);
      NM_STORE(0, 0)
      __syncthreads();
    }
    if (t < nk) {   // odd step count: the last step is in stage 0
      NM_COMPUTE(0)
    }
  }
#undef NM_KOFF
#undef NM_LOAD
#undef NM_STORE
#undef NM_COMPUTE
#undef NM_FRAGS
#undef NM_MMA
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * TM + i * 16 + 4 * lk + v;
        const int gn = n0 + wn * TN + j * 16 + lr;
        if (gm < M && gn < N) {
          double* c = C + (int64_t)gm * ldc + gn;
          const double r = alpha * (double)acc[i][j][v];
          *c = (beta == 0.0) ? r : r + beta * (*c);
        }
      }
}

// Output tile of each workgroup tile code of the split-precision GEMM (the
// codes are listed in kernels.h).
void bf16x3_tile_dims(int tile, int& bm, int& bn) {
  bm = (tile == 1 || tile == 2 || tile == 4 || tile == 6) ? 256 : 128;
  bn = (tile == 1 || tile == 3 || tile == 5 || tile == 7) ? 256 : 128;
}

// The shape used when none is given: the 128 x 128 kernel, measured faster
// than the one-workgroup-per-CU tiles on every shape timed so far (two
// workgroups per CU hide each other's load and barrier stalls); the large
// tiles stay available to the autotuner and nm_gemm_tiled.
int bf16x3_auto_tile(int M, int N, int batch) {
  (void)M;
  (void)N;
  (void)batch;
  return 0;
}

int gemm_bf16x3(hipStream_t s, int M, int N, int K, int batch, double alpha, const uint16_t* A,
                int64_t lda, int64_t sA, const uint16_t* B, int64_t ldb, int64_t sB, double beta,
                double* C, int64_t ldc, int64_t sC, int Klast, int tile) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  if (K <= 0 || K % HBK || (Klast > 0 && Klast % HBK) || lda % 8 || ldb % 8 || sA % 8 || sB % 8 ||
      lda < 2 * (int64_t)K || ldb < 2 * (int64_t)K || ((uintptr_t)A | (uintptr_t)B) % 16 ||
      tile >= kBf16Tiles)
    return -1;
  if (batch > 32768) {
    for (int b0 = 0; b0 < batch; b0 += 32768) {
      const int nb = batch - b0 < 32768 ? batch - b0 : 32768;
      int rc = gemm_bf16x3(s, M, N, K, nb, alpha, A + (int64_t)b0 * sA, lda, sA, B + (int64_t)b0 * sB, ldb,
                           sB, beta, C + (int64_t)b0 * sC, ldc, sC, b0 + nb == batch ? Klast : 0, tile);
      if (rc) return rc;
    }
    return 0;
  }
  if (tile < 0) tile = bf16x3_auto_tile(M, N, batch);
  int bm, bn;
  bf16x3_tile_dims(tile, bm, bn);
  dim3 grid((N + bn - 1) / bn, (M + bm - 1) / bm, batch);
#define NM_BF16BIG(BM_, BN_, WM_, WN_, PD_)                                                              \
  hipLaunchKernelGGL((gemm_bf16x3_big_kernel<BM_, BN_, WM_, WN_, PD_>), grid, dim3(WM_ * WN_ * 64), 0, s, \
                     M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast)
  switch (tile) {
    case 1: NM_BF16BIG(256, 256, 2, 4, 1); break;
    case 2: NM_BF16BIG(256, 128, 4, 2, 1); break;
    case 3: NM_BF16BIG(128, 256, 2, 4, 1); break;
    case 4: NM_BF16BIG(256, 128, 4, 2, 2); break;
    case 5: NM_BF16BIG(128, 256, 2, 4, 2); break;
    case 6: NM_BF16BIG(256, 128, 4, 2, 3); break;
    case 7: NM_BF16BIG(128, 256, 2, 4, 3); break;
    default:
      hipLaunchKernelGGL(gemm_bf16x3_kernel, grid, dim3(512), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB,
                         beta, C, ldc, sC, Klast);
  }
#undef NM_BF16BIG
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// fp32 -> bfloat16, rounded to nearest even (pairs: hi = bf16(x),
// lo = bf16(x - hi))
__device__ inline uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Position of the hi half of planar pair element p in an interleaved pair
// array (rows of Kp elements, Kp a multiple of 8): the 8-element chunk of p
// becomes 16 elements, hi first; its lo half sits 8 further.
__device__ inline int64_t pair_index(int64_t p) { return 2 * p - (p & 7); }

// ------------------------------------------------------ tiled strided copy
// A strided copy without summed labels runs as 64 x 64 tiles of two of its
// dimensions: X, the input's fastest, and Y, the output's fastest; every
// other dimension is a batch index decoded once per workgroup.  When X != Y
// the tile passes through LDS (row stride 65 doubles: the transposed reads of
// one wave fall in distinct banks), so loads run along X and stores along Y,
// both coalesced.  When X == Y, Y is the output's next-fastest dimension and
// each lane stores what it loaded.
struct TileSpec {
  int64_t nx = 1, ny = 1, isx = 0, isy = 0, osx = 0, osy = 0;
  int64_t tx = 1, ty = 1;
  int nb = 0;
  int64_t bdims[kMaxViewDims] = {0}, bistr[kMaxViewDims] = {0}, bostr[kMaxViewDims] = {0};
};

// Threads per 64 x 64 tile: eight waves, eight rows or columns of the tile
// per pass (measured against four waves: 20-50 % more bandwidth for the
// transposing copy, which also loads the old output values of a beta update
// before the LDS round trip, and 5-14 % for the direct one).
constexpr int kTileThreads = 512;

// PAIR: out is a bfloat16 pair array (uint16) whose planar position p (the
// output strides address a [rows][Kp] plane, p counted from pbase) is stored
// interleaved: hi at 2 p - p % 8, lo 8 further (pair_index); x = (float)(alpha
// in), hi = bf16(x), lo = bf16(x - hi)
template <typename TO, bool TRANS, bool PAIR = false>
__global__ __launch_bounds__(kTileThreads) void tile_copy_kernel(TO* __restrict__ out,
                                                                const double* __restrict__ in,
                                                                TileSpec t, double alpha, double beta,
                                                                int64_t pbase = 0) {
  __shared__ double tile[TRANS ? 64 * 65 : 1];
  int64_t b = blockIdx.x;
  const int64_t txi = b % t.tx;
  b /= t.tx;
  const int64_t tyi = b % t.ty;
  b /= t.ty;
  int64_t ib = 0, ob = 0;
  for (int d = t.nb - 1; d >= 0; --d) {
    const int64_t q = b / t.bdims[d];
    const int64_t i = b - q * t.bdims[d];
    b = q;
    ib += i * t.bistr[d];
    ob += i * t.bostr[d];
  }
  constexpr int RP = kTileThreads / 64, NI = 64 / RP;
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int64_t x0 = txi * 64, y0 = tyi * 64;
  if constexpr (TRANS) {
    // lanes along X for the loads, along Y for the stores; pass k of this
    // thread covers tile row (load) or column (store) row + RP k
    double prev[NI];
    if (!PAIR && beta != 0.0) {
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int64_t y = y0 + lane, x = x0 + row + RP * k;
        prev[k] = (x < t.nx && y < t.ny) ? (double)out[ob + x * t.osx + y * t.osy] : 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int64_t x = x0 + lane, y = y0 + row + RP * k;
      if (x < t.nx && y < t.ny) tile[(row + RP * k) * 65 + lane] = in[ib + x * t.isx + y * t.isy];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int64_t y = y0 + lane, x = x0 + row + RP * k;
      if (x < t.nx && y < t.ny) {
        const double val = alpha * tile[lane * 65 + row + RP * k];
        if constexpr (PAIR) {
          const float xf = (float)val;
          const uint16_t h = bf16_rne(xf);
          TO* o = out + pair_index(pbase + ob + x * t.osx + y * t.osy);
          o[0] = h;
          o[8] = bf16_rne(xf - __uint_as_float((uint32_t)h << 16));
        } else {
          TO* o = out + ob + x * t.osx + y * t.osy;
          *o = (beta == 0.0) ? (TO)val : (TO)(val + beta * prev[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int r = row; r < 64; r += RP) {
      const int64_t x = x0 + lane, y = y0 + r;
      if (x < t.nx && y < t.ny) {
        const double val = alpha * in[ib + x * t.isx + y * t.isy];
        if constexpr (PAIR) {
          const float xf = (float)val;
          const uint16_t h = bf16_rne(xf);
          TO* o = out + pair_index(pbase + ob + x * t.osx + y * t.osy);
          o[0] = h;
          o[8] = bf16_rne(xf - __uint_as_float((uint32_t)h << 16));
        } else {
          TO* o = out + ob + x * t.osx + y * t.osy;
          *o = (beta == 0.0) ? (TO)val : (TO)(val + beta * (double)*o);
        }
      }
    }
  }
}

// Plans a tiled copy for `v`; false when the view has summed labels or the
// tiles would be mostly empty (the generic kernel then runs).
static bool plan_tiles(const ViewSpec& v, TileSpec& t, bool& trans) {
  if (v.nr != 0) return false;
  int nd = 0;
  int64_t dims[kMaxViewDims], is[kMaxViewDims], os[kMaxViewDims];
  for (int d = 0; d < v.nd; ++d) {
    if (v.dims[d] == 1) continue;
    // merge with the previous kept dimension when both maps nest
    if (nd > 0 && is[nd - 1] == v.istr[d] * v.dims[d] && os[nd - 1] == v.ostr[d] * v.dims[d]) {
      dims[nd - 1] *= v.dims[d];
      is[nd - 1] = v.istr[d];
      os[nd - 1] = v.ostr[d];
      continue;
    }
    dims[nd] = v.dims[d];
    is[nd] = v.istr[d];
    os[nd] = v.ostr[d];
    ++nd;
  }
  if (nd < 2) return false;
  int X = 0, Y = 0;
  for (int d = 1; d < nd; ++d) {
    if (is[d] < is[X]) X = d;
    if (os[d] < os[Y]) Y = d;
  }
  trans = X != Y;
  if (!trans) {
    Y = -1;
    for (int d = 0; d < nd; ++d)
      if (d != X && (Y < 0 || os[d] < os[Y])) Y = d;
  }
  t.nx = dims[X];
  t.isx = is[X];
  t.osx = os[X];
  t.ny = dims[Y];
  t.isy = is[Y];
  t.osy = os[Y];
  t.tx = (t.nx + 63) / 64;
  t.ty = (t.ny + 63) / 64;
  t.nb = 0;
  int64_t nbatch = 1;
  for (int d = 0; d < nd; ++d) {
    if (d == X || d == Y) continue;
    t.bdims[t.nb] = dims[d];
    t.bistr[t.nb] = is[d];
    t.bostr[t.nb] = os[d];
    ++t.nb;
    nbatch *= dims[d];
  }
  const double fill = (double)(t.nx * t.ny) / (double)(t.tx * 64 * t.ty * 64);
  const double blocks = (double)t.tx * (double)t.ty * (double)nbatch;
  return fill >= 1.0 / 16.0 && blocks < (double)(1 << 24);
}

template <typename TO>
static int tile_copy(hipStream_t s, TO* out, const double* in, const ViewSpec& v, double alpha,
                     double beta) {
  TileSpec t;
  bool trans = false;
  if (!plan_tiles(v, t, trans)) return 1;
  int64_t blocks = t.tx * t.ty;
  for (int d = 0; d < t.nb; ++d) blocks *= t.bdims[d];
  if (trans)
    hipLaunchKernelGGL((tile_copy_kernel<TO, true>), dim3((unsigned)blocks), dim3(kTileThreads), 0,
                       s, out + v.obase, in + v.ibase, t, alpha, beta);
  else
    hipLaunchKernelGGL((tile_copy_kernel<TO, false>), dim3((unsigned)blocks), dim3(kTileThreads), 0,
                       s, out + v.obase, in + v.ibase, t, alpha, beta);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// out (float) = in (double) through a strided view (packing for the fp32 path)
__global__ void view_gather_f32_kernel(float* __restrict__ out, const double* __restrict__ in,
                                       ViewSpec v, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, oo = v.obase, io = v.ibase;
    for (int d = v.nd - 1; d >= 0; --d) {
      const int64_t q = rem / v.dims[d];
      const int64_t i = rem - q * v.dims[d];
      rem = q;
      oo += i * v.ostr[d];
      io += i * v.istr[d];
    }
    out[oo] = (float)in[io];
  }
}

__global__ void flat_f32_kernel(float* __restrict__ out, const double* __restrict__ in, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (float)in[e];
}

int view_gather_f32(hipStream_t s, float* out, const double* in, const ViewSpec& v) {
  int64_t total = 1;
  for (int d = 0; d < v.nd; ++d) total *= v.dims[d];
  if (total == 0) return 0;
  // a contiguous view in its own order: an elementwise conversion
  bool flat = true;
  int64_t st = 1;
  for (int d = v.nd - 1; d >= 0; --d) {
    if (v.dims[d] != 1 && (v.istr[d] != st || v.ostr[d] != st)) flat = false;
    st *= v.dims[d];
  }
  if (flat) {
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(flat_f32_kernel, dim3((int)g), dim3(256), 0, s, out + v.obase, in + v.ibase, total);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  const int rc = tile_copy<float>(s, out, in, v, 1.0, 0.0);
  if (rc <= 0) return rc;
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(view_gather_f32_kernel, dim3((int)g), dim3(256), 0, s, out, in, v, total);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// bfloat16 pair of in (double) through a strided view into an interleaved
// pair array (generic path when the view does not tile)
__global__ void view_gather_bf16x2_kernel(uint16_t* __restrict__ out, const double* __restrict__ in,
                                          ViewSpec v, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, oo = v.obase, io = v.ibase;
    for (int d = v.nd - 1; d >= 0; --d) {
      const int64_t q = rem / v.dims[d];
      const int64_t i = rem - q * v.dims[d];
      rem = q;
      oo += i * v.ostr[d];
      io += i * v.istr[d];
    }
    const float xf = (float)in[io];
    const uint16_t h = bf16_rne(xf);
    uint16_t* o = out + pair_index(oo);
    o[0] = h;
    o[8] = bf16_rne(xf - __uint_as_float((uint32_t)h << 16));
  }
}

// planar positions pbase + e, e < total, from in[e]
__global__ void flat_bf16x2_kernel(uint16_t* __restrict__ out, int64_t pbase,
                                   const double* __restrict__ in, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float xf = (float)in[e];
    const uint16_t h = bf16_rne(xf);
    uint16_t* o = out + pair_index(pbase + e);
    o[0] = h;
    o[8] = bf16_rne(xf - __uint_as_float((uint32_t)h << 16));
  }
}

// zero the padding columns [K, Kp) of a [rows][Kp] pair plane
__global__ void pad_bf16x2_kernel(uint16_t* __restrict__ out, int64_t rows, int K, int Kp) {
  const int w = Kp - K;
  const int64_t total = rows * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w;
    uint16_t* o = out + pair_index(r * Kp + K + (e - r * w));
    o[0] = 0;
    o[8] = 0;
  }
}

int view_gather_bf16x2(hipStream_t s, uint16_t* out, const double* in, const ViewSpec& v, int64_t rows,
                       int K, int Kp) {
  if (Kp % 8) return -1;
  int64_t total = 1;
  for (int d = 0; d < v.nd; ++d) total *= v.dims[d];
  // a contiguous view in its own order (no permutation, no padding): an
  // elementwise pass
  bool flat = true;
  int64_t st = 1;
  for (int d = v.nd - 1; d >= 0; --d) {
    if (v.dims[d] != 1 && (v.istr[d] != st || v.ostr[d] != st)) flat = false;
    st *= v.dims[d];
  }
  if (total > 0 && flat) {
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(flat_bf16x2_kernel, dim3((int)g), dim3(256), 0, s, out, v.obase, in + v.ibase,
                       total);
    if (hipGetLastError() != hipSuccess) return -3;
  } else if (total > 0) {
    TileSpec t;
    bool trans = false;
    if (plan_tiles(v, t, trans)) {
      int64_t blocks = t.tx * t.ty;
      for (int d = 0; d < t.nb; ++d) blocks *= t.bdims[d];
      if (trans)
        hipLaunchKernelGGL((tile_copy_kernel<uint16_t, true, true>), dim3((unsigned)blocks),
                           dim3(kTileThreads), 0, s, out, in + v.ibase, t, 1.0, 0.0, v.obase);
      else
        hipLaunchKernelGGL((tile_copy_kernel<uint16_t, false, true>), dim3((unsigned)blocks),
                           dim3(kTileThreads), 0, s, out, in + v.ibase, t, 1.0, 0.0, v.obase);
    } else {
      int64_t g = (total + 255) / 256;
      if (g > 65536) g = 65536;
      hipLaunchKernelGGL(view_gather_bf16x2_kernel, dim3((int)g), dim3(256), 0, s, out, in, v, total);
    }
    if (hipGetLastError() != hipSuccess) return -3;
  }
  if (Kp > K && rows > 0) {
    int64_t g = (rows * (Kp - K) + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(pad_bf16x2_kernel, dim3((int)g), dim3(256), 0, s, out, rows, K, Kp);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  return 0;
}

int gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, int batch, double alpha,
             const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb,
             int64_t sB, double beta, double* C, int64_t ldc, int64_t sC, int Klast) {
  if (M <= 0 || N <= 0 || batch <= 0) return 0;
  if (K <= 0) {  // C = beta C
    return -1;
  }
  if (batch > 32768) {   // grid.z limit: launch in chunks
    for (int b0 = 0; b0 < batch; b0 += 32768) {
      const int nb = batch - b0 < 32768 ? batch - b0 : 32768;
      int rc = gemm_f64(s, ta, tb, M, N, K, nb, alpha, A + (int64_t)b0 * sA, lda, sA,
                        B + (int64_t)b0 * sB, ldb, sB, beta, C + (int64_t)b0 * sC, ldc, sC,
                        b0 + nb == batch ? Klast : 0);
      if (rc) return rc;
    }
    return 0;
  }
  if (M >= LBM && N >= LBN) {
    dim3 grid((N + LBN - 1) / LBN, (M + LBM - 1) / LBM, batch);
#define NM_BIG(TA_, TB_, NT_) \
  hipLaunchKernelGGL((gemm_f64_big_kernel<TA_, TB_, NT_>), grid, dim3(NT_), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast)
    // 512 threads (2 workgroups of 8 waves per CU) measured 1.4x faster than
    // 256 threads with 64 x 64 per wave on the FP64 ladder and ring shapes.
    if (!ta && !tb) NM_BIG(false, false, 512);
    else if (!ta && tb) NM_BIG(false, true, 512);
    else if (ta && !tb) NM_BIG(true, false, 512);
    else NM_BIG(true, true, 512);
#undef NM_BIG
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  dim3 block(256);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, Klast);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ------------------------------------------------------------ strided views
// out[obase + sum_d i_d ostr_d] (=|+=) alpha * sum_red in[ibase + sum_d i_d istr_d
//                                                       + sum_r j_r rstr_r]
__global__ void view_gather_kernel(double* __restrict__ out, const double* __restrict__ in,
                                   ViewSpec v, double alpha, double beta, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, oo = v.obase, io = v.ibase;
    for (int d = v.nd - 1; d >= 0; --d) {
      const int64_t q = rem / v.dims[d];
      const int64_t i = rem - q * v.dims[d];
      rem = q;
      oo += i * v.ostr[d];
      io += i * v.istr[d];
    }
    double acc = 0.0;
    if (v.nr == 0) {
      acc = in[io];
    } else if (v.nr == 1) {
      for (int64_t j = 0; j < v.rdims[0]; ++j) acc += in[io + j * v.rstr[0]];
    } else {
      for (int64_t j0 = 0; j0 < v.rdims[0]; ++j0)
        for (int64_t j1 = 0; j1 < v.rdims[1]; ++j1)
          acc += in[io + j0 * v.rstr[0] + j1 * v.rstr[1]];
    }
    out[oo] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * out[oo];
  }
}

// in[ibase + ...] += alpha * out[obase + ...]; requires the map
// (i, j) -> input offset to be injective (no two threads hit one element).
__global__ void view_scatter_kernel(double* __restrict__ in, const double* __restrict__ out,
                                    ViewSpec v, double alpha, int64_t total) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, oo = v.obase, io = v.ibase;
    for (int d = v.nd - 1; d >= 0; --d) {
      const int64_t q = rem / v.dims[d];
      const int64_t i = rem - q * v.dims[d];
      rem = q;
      oo += i * v.ostr[d];
      io += i * v.istr[d];
    }
    const double val = alpha * out[oo];
    if (v.nr == 0) {
      in[io] += val;
    } else if (v.nr == 1) {
      for (int64_t j = 0; j < v.rdims[0]; ++j) in[io + j * v.rstr[0]] += val;
    } else {
      for (int64_t j0 = 0; j0 < v.rdims[0]; ++j0)
        for (int64_t j1 = 0; j1 < v.rdims[1]; ++j1)
          in[io + j0 * v.rstr[0] + j1 * v.rstr[1]] += val;
    }
  }
}

static int grid_for(int64_t total) {
  int64_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

int view_gather(hipStream_t s, double* out, const double* in, const ViewSpec& v, double alpha,
                double beta) {
  int64_t total = 1;
  for (int d = 0; d < v.nd; ++d) total *= v.dims[d];
  if (total == 0) return 0;
  const int rc = tile_copy<double>(s, out, in, v, alpha, beta);
  if (rc <= 0) return rc;
  hipLaunchKernelGGL(view_gather_kernel, dim3(grid_for(total)), dim3(256), 0, s, out, in, v,
                     alpha, beta, total);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int view_scatter(hipStream_t s, double* in, const double* out, const ViewSpec& v, double alpha) {
  int64_t total = 1;
  for (int d = 0; d < v.nd; ++d) total *= v.dims[d];
  if (total == 0) return 0;
  hipLaunchKernelGGL(view_scatter_kernel, dim3(grid_for(total)), dim3(256), 0, s, in, out, v,
                     alpha, total);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ------------------------------------------------------------- elementwise
__global__ void fill_kernel(double* x, double val, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = val;
}

int fill(hipStream_t s, double* x, double val, int64_t n) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, val, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// y = a x + b y
__global__ void axpby_kernel(double* y, const double* x, double a, double b, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (b == 0.0) ? a * x[e] : a * x[e] + b * y[e];
}

// dst[r ldd + j] = src[r lds + j] for j < len, row r = blockIdx.y (+ r0):
// four independent loads per thread in flight
__global__ __launch_bounds__(256) void rows_copy_kernel(double* __restrict__ dst, int64_t ldd,
                                                        const double* __restrict__ src, int64_t lds,
                                                        int64_t len) {
  const int64_t r = blockIdx.y;
  const double* a = src + r * lds;
  double* d = dst + r * ldd;
  for (int64_t j0 = (int64_t)blockIdx.x * 1024 + threadIdx.x; j0 < len; j0 += (int64_t)gridDim.x * 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = j0 + 256 * u < len ? a[j0 + 256 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + 256 * u < len) d[j0 + 256 * u] = v[u];
  }
}

int rows_copy(hipStream_t s, double* dst, int64_t ldd, const double* src, int64_t lds, int64_t len,
              int64_t rows) {
  if (len <= 0 || rows <= 0) return 0;
  const unsigned gx = (unsigned)std::min<int64_t>((len + 1023) / 1024, 8192);
  for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
    const int64_t rr = std::min<int64_t>(65535, rows - r0);
    hipLaunchKernelGGL(rows_copy_kernel, dim3(gx, (unsigned)rr), dim3(256), 0, s, dst + r0 * ldd, ldd,
                       src + r0 * lds, lds, len);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int axpby(hipStream_t s, double* y, const double* x, double a, double b, int64_t n) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, b, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Amplitude-shaped vector: [o*v singles][o*o*v*v doubles t2[i][j][a][b]].
// y = x / (shift - D) with D the orbital-energy difference (preconditioner);
// the sign convention: mode 0 -> y = -x / D (Jacobi step), mode 1 -> y = x / (shift - D).
__global__ void denom_kernel(double* y, const double* x, const double* eps, int o, int v,
                             double shift, int mode, double floor_abs) {
  const int64_t nov = (int64_t)o * v, n2 = nov * nov;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nov + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    double D;
    if (e < nov) {
      const int i = (int)(e / v), a = (int)(e % v);
      D = eps[o + a] - eps[i];
    } else {
      int64_t r = e - nov;
      const int b = (int)(r % v); r /= v;
      const int a = (int)(r % v); r /= v;
      const int j = (int)(r % o);
      const int i = (int)(r / o);
      D = eps[o + a] + eps[o + b] - eps[i] - eps[j];
    }
    double d = (mode == 0) ? -D : shift - D;
    if (fabs(d) < floor_abs) d = (d < 0.0) ? -floor_abs : floor_abs;
    y[e] = x[e] / d;
  }
}

int apply_denominator(hipStream_t s, double* y, const double* x, const double* eps, int o,
                      int v, double shift, int mode) {
  const int64_t n = (int64_t)o * v * (1 + (int64_t)o * v);
  hipLaunchKernelGGL(denom_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, eps, o, v, shift,
                     mode, 1e-3);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Half layout of an amplitude-shaped vector: the singles, then the doubles
// x2[i][j][a][b] of the unordered pairs P = i v + a <= Q = j v + b, row by
// row of the upper triangle (offset P nov - P (P - 1) / 2 + Q - P).  For
// vectors with x2[i][j][a][b] = x2[j][i][b][a] the biorthonormal product is
// the plain dot product of their half layouts.
__device__ inline int64_t half_index(int64_t P, int64_t Q, int64_t nov) {
  return nov + P * nov - P * (P - 1) / 2 + (Q - P);
}

// full (symmetric doubles) -> half; one thread per full element, the P <= Q
// ones write (contiguously in Q for a fixed P)
__global__ void half_pack_kernel(double* __restrict__ h, const double* __restrict__ x, int o, int v) {
  const int64_t nov = (int64_t)o * v, n2 = nov * nov;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nov + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nov) {
      h[e] = x[e];
      continue;
    }
    int64_t r = e - nov;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const int64_t P = (int64_t)i * v + a, Q = (int64_t)j * v + b;
    if (P <= Q) h[half_index(P, Q, nov)] = x[e];
  }
}

// half -> full symmetric doubles
__global__ void half_unpack_kernel(double* __restrict__ x, const double* __restrict__ h, int o, int v) {
  const int64_t nov = (int64_t)o * v, n2 = nov * nov;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nov + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nov) {
      x[e] = h[e];
      continue;
    }
    int64_t r = e - nov;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const int64_t P = (int64_t)i * v + a, Q = (int64_t)j * v + b;
    x[e] = P <= Q ? h[half_index(P, Q, nov)] : h[half_index(Q, P, nov)];
  }
}

// y = x / (shift - D) on the half layout (D the orbital-energy difference of
// the element; |shift - D| kept >= floor_abs), as denom_kernel's mode 1
__global__ void half_denom_kernel(double* y, const double* x, const double* eps, int o, int v,
                                  double shift, double floor_abs) {
  const int64_t nov = (int64_t)o * v, nh = nov + nov * (nov + 1) / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nh;
       e += (int64_t)gridDim.x * blockDim.x) {
    double D;
    if (e < nov) {
      const int i = (int)(e / v), a = (int)(e % v);
      D = eps[o + a] - eps[i];
    } else {
      // row P of the upper triangle: the largest P with its offset <= e - nov
      const int64_t t = e - nov;
      const double nn = (double)nov;
      int64_t P = (int64_t)(((2.0 * nn + 1.0) - sqrt((2.0 * nn + 1.0) * (2.0 * nn + 1.0) - 8.0 * (double)t)) * 0.5);
      if (P < 0) P = 0;
      if (P > nov - 1) P = nov - 1;
      while (P > 0 && P * nov - P * (P - 1) / 2 > t) --P;
      while (P + 1 < nov && (P + 1) * nov - (P + 1) * P / 2 <= t) ++P;
      const int64_t Q = P + (t - (P * nov - P * (P - 1) / 2));
      const int i = (int)(P / v), a = (int)(P % v), j = (int)(Q / v), b = (int)(Q % v);
      D = eps[o + a] + eps[o + b] - eps[i] - eps[j];
    }
    double d = shift - D;
    if (fabs(d) < floor_abs) d = (d < 0.0) ? -floor_abs : floor_abs;
    y[e] = x[e] / d;
  }
}

int half_pack(hipStream_t s, double* h, const double* x, int o, int v) {
  const int64_t n = (int64_t)o * v * (1 + (int64_t)o * v);
  hipLaunchKernelGGL(half_pack_kernel, dim3(grid_for(n)), dim3(256), 0, s, h, x, o, v);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int half_unpack(hipStream_t s, double* x, const double* h, int o, int v) {
  const int64_t n = (int64_t)o * v * (1 + (int64_t)o * v);
  hipLaunchKernelGGL(half_unpack_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, h, o, v);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int half_denominator(hipStream_t s, double* y, const double* x, const double* eps, int o, int v,
                     double shift) {
  const int64_t nov = (int64_t)o * v, n = nov + nov * (nov + 1) / 2;
  hipLaunchKernelGGL(half_denom_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, eps, o, v, shift,
                     1e-3);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Packed-metric weights on the doubles block: w = 1/2 (1 + delta_(ia),(jb)).
// mode 0: y = w x (seed of a packed functional on the full tensor);
// mode 1: y[ijab] = x[ijab] + x[jiba] - delta x (full-tensor gradient -> packed gradient);
// mode 2: y <- symmetric part of y in place (x unused): keeps vectors in the
//         space of doubles with x2[i][j][a][b] == x2[j][i][b][a].
__global__ void metric_kernel(double* y, const double* x, int o, int v, int mode) {
  const int64_t nov = (int64_t)o * v, n2 = nov * nov;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nov + n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nov) {
      if (mode != 2) y[e] = x[e];
      continue;
    }
    int64_t r = e - nov;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const bool diag = (i == j) && (a == b);
    if (mode == 2) {  // in place: x2 <- (x2 + x2^T)/2, one thread per unordered pair
      const int64_t P = (int64_t)i * v + a, Q = (int64_t)j * v + b;
      if (P < Q) {
        const int64_t t = nov + (((int64_t)j * o + i) * v + b) * v + a;
        const double m = 0.5 * (y[e] + y[t]);
        y[e] = m;
        y[t] = m;
      }
      continue;
    }
    if (mode == 0) {
      y[e] = diag ? x[e] : 0.5 * x[e];
    } else {
      const int64_t t = nov + (((int64_t)j * o + i) * v + b) * v + a;
      y[e] = diag ? x[e] : x[e] + x[t];
    }
  }
}

int apply_metric(hipStream_t s, double* y, const double* x, int o, int v, int mode) {
  const int64_t n = (int64_t)o * v * (1 + (int64_t)o * v);
  hipLaunchKernelGGL(metric_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, o, v, mode);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// --------------------------------------------------------------- reductions
// Pass 1: per-block partial sums (wavefront shuffles, then LDS across waves).
__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
__device__ inline double wave_max(double x) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
  return x;
}

// Packed-metric dot: sum singles + 1/2 sum doubles + 1/2 sum diagonal doubles
// when `packed` != 0 (amplitude-shaped vectors), plain dot otherwise.
__global__ __launch_bounds__(256) void dot_partial_kernel(const double* x, const double* y,
                                                          int64_t n, int o, int v, int packed,
                                                          double* part) {
  __shared__ double red[4];
  double acc = 0.0;
  const int64_t nov = (int64_t)o * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double w = 1.0;
    if (packed && e >= nov) {
      int64_t r = e - nov;
      const int b = (int)(r % v); r /= v;
      const int a = (int)(r % v); r /= v;
      const int j = (int)(r % o);
      const int i = (int)(r / o);
      w = (i == j && a == b) ? 1.0 : 0.5;
    }
    acc += w * x[e] * y[e];
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void absmax_partial_kernel(const double* x, int64_t n,
                                                             double* part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double a = fabs(x[e]);
    // a NaN counts as +inf: the max reductions below (fmax) would drop it
    acc = (a != a) ? INFINITY : (a > acc ? a : acc);
  }
  acc = wave_max(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Pass 2: one block folds the partials (fixed order: deterministic).
__global__ __launch_bounds__(256) void fold_kernel(const double* part, int np, int op,
                                                   double* out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int e = threadIdx.x; e < np; e += 256) acc = op ? fmax(acc, part[e]) : acc + part[e];
  acc = op ? wave_max(acc) : wave_sum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    *out = op ? fmax(fmax(red[0], red[1]), fmax(red[2], red[3]))
              : red[0] + red[1] + red[2] + red[3];
}

constexpr int kReduceBlocks = 1024;

int dot(hipStream_t s, const double* x, const double* y, int64_t n, int o, int v, int packed,
        double* scratch, double* out_dev) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kReduceBlocks), dim3(256), 0, s, x, y, n, o, v,
                     packed, scratch);
  hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(256), 0, s, scratch, kReduceBlocks, 0, out_dev);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int absmax(hipStream_t s, const double* x, int64_t n, double* scratch, double* out_dev) {
  hipLaunchKernelGGL(absmax_partial_kernel, dim3(kReduceBlocks), dim3(256), 0, s, x, n, scratch);
  hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(256), 0, s, scratch, kReduceBlocks, 1, out_dev);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int reduce_scratch_doubles() { return kReduceBlocks; }

// ------------------------------------------------------- multi-row vectors
// out[k] = sum_e V[k][e] x[e] for the m <= kMaxRows rows of V (row-major,
// row stride n).  Every block covers a contiguous chunk of e, reads x once and
// keeps m partial sums per thread; partials [block][k] are folded in a fixed
// order by a second kernel (deterministic).  1024 blocks of 4 waves: 16 waves
// per CU in flight, enough loads to cover HBM latency.
constexpr int kRowBlocks = 1024;

// out[r * m + k] = sum_b part[b * bstride + r * kMaxRows + k]: one workgroup
// per output, fixed-order strided sums and a fixed tree (deterministic).
__global__ __launch_bounds__(256) void rows_fold_par_kernel(const double* __restrict__ part, int nb,
                                                            int m, int64_t bstride,
                                                            double* __restrict__ out) {
  __shared__ double red[256];
  const int o = blockIdx.x, r = o / m, k = o % m;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[(int64_t)b * bstride + r * kMaxRows + k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = red[0];
}

constexpr int kRowGroup = 8;   // rows accumulated in registers at a time

__global__ __launch_bounds__(256) void rows_dot_partial_kernel(const double* __restrict__ V,
                                                               int m, int64_t n,
                                                               const double* __restrict__ x,
                                                               double* part) {
  __shared__ double red[4][kRowGroup];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = blockIdx.x * chunk;
  const int64_t e1 = e0 + chunk < n ? e0 + chunk : n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int g0 = 0; g0 < m; g0 += kRowGroup) {
    double acc[kRowGroup];
#pragma unroll
    for (int k = 0; k < kRowGroup; ++k) acc[k] = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const double xe = x[e];
#pragma unroll
      for (int k = 0; k < kRowGroup; ++k)
        if (g0 + k < m) acc[k] += V[(int64_t)(g0 + k) * n + e] * xe;
    }
#pragma unroll
    for (int k = 0; k < kRowGroup; ++k) {
      double a = acc[k];
      for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
      if (lane == 0) red[wid][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < kRowGroup && g0 + threadIdx.x < m) {
      const int k = threadIdx.x;
      part[(int64_t)blockIdx.x * kMaxRows + g0 + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    }
    __syncthreads();
  }
}

int rows_dot(hipStream_t s, const double* V, int m, int64_t n, const double* x, double* part,
             double* out) {
  if (m <= 0) return 0;
  if (m > kMaxRows) return -1;
  hipLaunchKernelGGL(rows_dot_partial_kernel, dim3(kRowBlocks), dim3(256), 0, s, V, m, n, x, part);
  hipLaunchKernelGGL(rows_fold_par_kernel, dim3(m), dim3(256), 0, s, part, kRowBlocks, m,
                     (int64_t)kMaxRows, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int rows_scratch_doubles() { return kRowBlocks * kMaxRows * kMaxRhs; }

// Several right-hand sides at once (R <= kMaxRhs vectors X[r] = X + r ldx):
// part[b][r][k] = sum over block b's chunk of V[k][e] X[r][e]; every row of V
// is read once for all R vectors.
template <int R>
__global__ __launch_bounds__(256) void rows_dot_multi_partial_kernel(
    const double* __restrict__ V, int m, int64_t n, const double* __restrict__ X, int64_t ldx,
    double* part) {
  __shared__ double red[4][R][kRowGroup];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = blockIdx.x * chunk;
  const int64_t e1 = e0 + chunk < n ? e0 + chunk : n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int g0 = 0; g0 < m; g0 += kRowGroup) {
    double acc[R][kRowGroup];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < kRowGroup; ++k) acc[r][k] = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      double xe[R];
#pragma unroll
      for (int r = 0; r < R; ++r) xe[r] = X[(int64_t)r * ldx + e];
#pragma unroll
      for (int k = 0; k < kRowGroup; ++k)
        if (g0 + k < m) {
          const double vk = V[(int64_t)(g0 + k) * n + e];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r][k] += vk * xe[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < kRowGroup; ++k) {
        double a = acc[r][k];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[wid][r][k] = a;
      }
    __syncthreads();
    if (threadIdx.x < R * kRowGroup) {
      const int r = threadIdx.x / kRowGroup, k = threadIdx.x % kRowGroup;
      if (g0 + k < m)
        part[((int64_t)blockIdx.x * kMaxRhs + r) * kMaxRows + g0 + k] =
            red[0][r][k] + red[1][r][k] + red[2][r][k] + red[3][r][k];
    }
    __syncthreads();
  }
}

int rows_dot_multi(hipStream_t s, const double* V, int m, int64_t n, const double* X, int64_t ldx,
                   int R, double* part, double* out) {
  if (m <= 0 || R <= 0) return 0;
  if (m > kMaxRows || R > kMaxRhs) return -1;
#define NM_RD(RR) \
  hipLaunchKernelGGL(rows_dot_multi_partial_kernel<RR>, dim3(kRowBlocks), dim3(256), 0, s, V, m, n, X, ldx, part)
  switch (R) {
    case 1: NM_RD(1); break;
    case 2: NM_RD(2); break;
    case 3: NM_RD(3); break;
    default: NM_RD(4); break;
  }
#undef NM_RD
  hipLaunchKernelGGL(rows_fold_par_kernel, dim3(R * m), dim3(256), 0, s, part, kRowBlocks, m,
                     (int64_t)kMaxRhs * kMaxRows, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// X[r][e] += alpha * sum_k H[r][k] V[k][e] for R vectors (H [R][m] on the
// device); every row of V is read once for all R vectors.
template <int R>
__global__ __launch_bounds__(256) void rows_axpy_multi_kernel(const double* __restrict__ V, int m,
                                                              int64_t n, const double* __restrict__ H,
                                                              double alpha, double* __restrict__ X,
                                                              int64_t ldx, int overwrite) {
  __shared__ double hs[R][kMaxRows];
  for (int t = threadIdx.x; t < R * m; t += blockDim.x) hs[t / m][t % m] = H[t];
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int k = 0; k < m; ++k) {
      const double vk = V[(int64_t)k * n + e];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += hs[r][k] * vk;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double* xr = X + (int64_t)r * ldx + e;
      *xr = overwrite ? alpha * acc[r] : *xr + alpha * acc[r];
    }
  }
}

int rows_axpy_multi(hipStream_t s, const double* V, int m, int64_t n, const double* H, double alpha,
                    double* X, int64_t ldx, int R, bool overwrite) {
  if (m <= 0 || R <= 0) return 0;
  if (m > kMaxRows || R > kMaxRhs) return -1;
#define NM_RA(RR) \
  hipLaunchKernelGGL(rows_axpy_multi_kernel<RR>, dim3(grid_for(n)), dim3(256), 0, s, V, m, n, H, alpha, X, ldx, (int)overwrite)
  switch (R) {
    case 1: NM_RA(1); break;
    case 2: NM_RA(2); break;
    case 3: NM_RA(3); break;
    default: NM_RA(4); break;
  }
#undef NM_RA
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// x[e] += alpha * sum_k h[k] V[k][e]   (h on the device)
__global__ __launch_bounds__(256) void rows_axpy_kernel(const double* __restrict__ V, int m,
                                                        int64_t n, const double* __restrict__ h,
                                                        double alpha, double* __restrict__ x) {
  __shared__ double hs[kMaxRows];
  if (threadIdx.x < m) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += hs[k] * V[(int64_t)k * n + e];
    x[e] += alpha * acc;
  }
}

int rows_axpy(hipStream_t s, const double* V, int m, int64_t n, const double* h, double alpha,
              double* x) {
  if (m <= 0) return 0;
  if (m > kMaxRows) return -1;
  hipLaunchKernelGGL(rows_axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, V, m, n, h, alpha, x);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace nm


