// Kernels of the blocked two-electron density (Sec. II C, eq. NAC_NC_densities):
// packing of symmetric index pairs, the vvvv block from its factors, and
// row-wise dot products for the per-direction contractions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace nm {

namespace {

// p >= q with p (p + 1) / 2 + q = j
__device__ inline void tri_decode(int64_t j, int& p, int& q) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)j + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > j) --r;
  while ((r + 1) * (r + 2) / 2 <= j) ++r;
  p = (int)r;
  q = (int)(j - r * (r + 1) / 2);
}

__global__ __launch_bounds__(256) void pack_pairs_kernel(const double* __restrict__ in, int64_t ldi,
                                                         int o, int v, int sum,
                                                         double* __restrict__ out, int64_t ldo) {
  const int n = o + v;
  const int64_t mo = (int64_t)o * (o + 1) / 2, mov = mo + (int64_t)o * v;
  const int64_t m = mov + (int64_t)v * (v + 1) / 2;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t r = blockIdx.y;
  int p, q;
  if (j < mo) {
    tri_decode(j, p, q);
  } else if (j < mov) {
    const int64_t k = j - mo;
    p = o + (int)(k % v);
    q = (int)(k / v);
  } else {
    tri_decode(j - mov, p, q);
    p += o;
    q += o;
  }
  const double* X = in + r * ldi;
  double val = X[(int64_t)p * n + q];
  if (sum && p != q) val += X[(int64_t)q * n + p];
  out[r * ldo + j] = val;
}

// One workgroup per packed row pair (a >= c), c in the chunk [c0, c0 + cc),
// and 32 x 32 tile of column pairs (b, d): the four index images of
// G[c][d][a][b] are read as rows of M1[x][y] = G[c][x][a][y] (from the chunk
// M1c[c - c0][x][a][y]) and M2[x][y] = G[a][x][c][y] (from
// M2c[a][x][c - c0][y]), y contiguous, and transposed through LDS so that the
// packed output (d fastest) is written in order.
__global__ __launch_bounds__(256) void pack_vvvv_rows_kernel(const double* __restrict__ M1c,
                                                             const double* __restrict__ M2c, int v,
                                                             int c0, int cc, int64_t mv,
                                                             double* __restrict__ out) {
  __shared__ double T[4][32][33];
  const int cl = blockIdx.y, c = c0 + cl, a = blockIdx.z;
  if (a < c) return;
  const int64_t r = (int64_t)a * (a + 1) / 2 + c;
  int tb, td;
  tri_decode(blockIdx.x, tb, td);
  const int b0 = tb * 32, d0 = td * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t v2 = (int64_t)v * v, s2 = (int64_t)cc * v;
  const double* M1 = M1c + (int64_t)cl * v * v2 + (int64_t)a * v;   // M1[x][y] = M1[x v2 + y]
  const double* M2 = M2c + (int64_t)a * v * s2 + (int64_t)cl * v;   // M2[x][y] = M2[x s2 + y]
  const bool two = (a != c);
  for (int i = ty; i < 32; i += 8) {
    const int d = d0 + i, b = b0 + i, bj = b0 + tx, dj = d0 + tx;
    const bool in0 = d < v && bj < v, in1 = b < v && dj < v;
    T[0][i][tx] = in0 ? M1[(int64_t)d * v2 + bj] : 0.0;
    T[1][i][tx] = in1 ? M1[(int64_t)b * v2 + dj] : 0.0;
    T[2][i][tx] = (two && in0) ? M2[(int64_t)d * s2 + bj] : 0.0;
    T[3][i][tx] = (two && in1) ? M2[(int64_t)b * s2 + dj] : 0.0;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int b = b0 + i, d = d0 + tx;
    if (b >= v || d > b) continue;
    // M1[d][b] = T[0][d - d0][b - b0], M1[b][d] = T[1][b - b0][d - d0]
    double s = T[0][tx][i] + T[2][tx][i];
    if (b != d) s += T[1][i][tx] + T[3][i][tx];
    out[r * mv + (int64_t)b * (b + 1) / 2 + d] = s;
  }
}

__global__ __launch_bounds__(256) void rowdot_kernel(const double* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb,
                                                     int64_t len, double alpha, double beta,
                                                     double* __restrict__ out) {
  const int64_t r = blockIdx.x;
  const double* a = A + r * lda;
  const double* b = B + r * ldb;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < len; j += blockDim.x) s += a[j] * b[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = part[0] + part[1] + part[2] + part[3];
    out[r] = alpha * t + (beta == 0.0 ? 0.0 : beta * out[r]);
  }
}

}  // namespace

int pack_pairs(hipStream_t s, double* out, int64_t ldo, const double* in, int64_t ldi, int64_t rows,
               int o, int v, bool sum) {
  if (rows <= 0) return 0;
  const int64_t m = (int64_t)(o + v) * (o + v + 1) / 2;
  for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
    const int64_t rr = std::min<int64_t>(65535, rows - r0);
    hipLaunchKernelGGL(pack_pairs_kernel, dim3((unsigned)((m + 255) / 256), (unsigned)rr), dim3(256),
                       0, s, in + r0 * ldi, ldi, o, v, sum ? 1 : 0, out + r0 * ldo, ldo);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int pack_vvvv_rows(hipStream_t s, double* out, const double* M1c, const double* M2c, int v, int c0,
                   int cc) {
  const int64_t mv = (int64_t)v * (v + 1) / 2;
  const int nt = (v + 31) / 32;
  if (cc <= 0 || c0 < 0 || c0 + cc > v || cc > 65535) return -1;
  hipLaunchKernelGGL(pack_vvvv_rows_kernel, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)cc, (unsigned)v),
                     dim3(256), 0, s, M1c, M2c, v, c0, cc, mv, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int rowdot(hipStream_t s, double* out, const double* A, int64_t lda, const double* B, int64_t ldb,
           int64_t rows, int64_t len, double alpha, double beta) {
  if (rows <= 0) return 0;
  if (rows > 0x7fffffffLL) return -1;
  hipLaunchKernelGGL(rowdot_kernel, dim3((unsigned)rows), dim3(256), 0, s, A, lda, B, ldb, len, alpha,
                     beta, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace nm
