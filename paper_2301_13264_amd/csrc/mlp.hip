// Learned initial guess: a three-layer SiLU perceptron trained and evaluated
// on the GPU with the library's own kernels.
//
// y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3,  s(u) = u / (1 + exp(-u)),
// weights row-major W[in][out].  The fp32 master parameters are updated by
// Adam; every product uses a working copy rounded to bfloat16 (round to
// nearest, ties to even), multiplied on the FP32 matrix cores with fp32
// accumulation (the products of bfloat16 values are exact in fp32).  The loss
// is half the mean squared error over all outputs.
//
// Memory per batch row: activations u1, h1, u2, h2 (fp32) and one fp64 GEMM
// output row of width entries; gradients of W reduce over the batch by split-K
// partial products folded in fp64.  Inference (mlp_forward) of the usual
// shapes runs instead as one fused kernel on the bf16 matrix cores that keeps
// every intermediate in registers (mlp_fused_kernel).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/nacme.h"
#include "kernels.h"

namespace nm {

__device__ inline float silu_f(float u) { return u / (1.0f + __expf(-u)); }
__device__ inline float silu_g(float u) {
  const float sg = 1.0f / (1.0f + __expf(-u));
  return sg * (1.0f + u * (1.0f - sg));
}
__device__ inline float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// u = acc + b (per column), h = s(u); acc fp64 [n][w]
__global__ void bias_act_kernel(const double* __restrict__ acc, const float* __restrict__ b,
                                float* __restrict__ u, float* __restrict__ h, int64_t n, int w,
                                int act) {
  const int64_t tot = n * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float x = (float)acc[e] + b[e % w];
    if (u) u[e] = x;
    h[e] = act ? silu_f(x) : x;
  }
}

// r = (y - t) / cnt written to dy; per-block partial sums of (y - t)^2
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ y,
                                                  const float* __restrict__ t,
                                                  float* __restrict__ dy, int64_t cnt,
                                                  double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[e] - t[e];
    dy[e] = r / (float)cnt;
    acc += (double)r * (double)r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// du = acc * s'(u)
__global__ void act_back_kernel(const double* __restrict__ acc, const float* __restrict__ u,
                                float* __restrict__ du, int64_t tot) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    du[e] = (float)acc[e] * silu_g(u[e]);
}

// column sums of x [n][w] over row chunks: part[chunk][col] (fp64)
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* __restrict__ x, int64_t n,
                                                             int w, int64_t rows_per_chunk,
                                                             double* __restrict__ part) {
  __shared__ double sh[4][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int lr = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  double acc = 0.0;
  if (col < w)
    for (int64_t r = r0 + lr; r < r1; r += 4) acc += (double)x[r * w + col];
  sh[lr][threadIdx.x & 63] = acc;
  __syncthreads();
  if (lr == 0 && col < w)
    part[(int64_t)blockIdx.y * w + col] =
        sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// out[e] = sum_z part[z][e] (fp32 result)
__global__ void fold_f32_kernel(const double* __restrict__ part, int nz, int64_t len,
                                float* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * len + e];
    out[e] = (float)s;
  }
}

// Adam on the master copy; the working copy is its bfloat16 rounding
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float* __restrict__ pw, int64_t np,
                            float lr, float c1, float c2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = 0.9f * m[e] + 0.1f * ge;
    const float ve = 0.999f * v[e] + 0.001f * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + 1e-8f);
    p[e] = pe;
    pw[e] = bf16_round(pe);
  }
}

__global__ void round_kernel(const float* __restrict__ p, float* __restrict__ pw, int64_t np) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np;
       e += (int64_t)gridDim.x * blockDim.x)
    pw[e] = bf16_round(p[e]);
}

// rows idx[k] of src [*][w] -> dst[k][w]
__global__ void gather_rows_kernel(const float* __restrict__ src, const int64_t* __restrict__ idx,
                                   int64_t k, int w, float* __restrict__ dst) {
  const int64_t tot = k * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / w;
    dst[e] = src[idx[r] * w + (e - r * w)];
  }
}

// ------------------------------------------------------ fused inference
// One pass of the whole network on the bf16 matrix cores, no intermediate
// rows in HBM: each wave takes 16 NS rows at a time (NS 16-row strips).
//   layer 1: u1^T = W1^T X^T (K = n_in <= 32, zero-padded), X carried as a
//            bfloat16 pair (hi + lo, about 2^-17 relative), W1 exact in bf16;
//   layer 2: u2 = h1 W2 with h1 = s(u1 + b1) as a bfloat16 pair, W2 exact;
//   layer 3: y = s(u2 + b2) W3 + b3 on the vector units, reduced across the
//            16 lanes that hold one row's columns.
// MFMA v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] (j < 8) and receives D[4 (l / 16) + v][l % 16]
// (v < 4).  Layer 1's output lands with lane l holding row l % 16 and hidden
// units 16 c + 4 (l / 16) + v of chunk c, which is already layer 2's A layout
// once the hidden index inside each 32-wide K block is taken in the order
//   kk = 8 g + j  <->  k = 32 kb + 16 (j / 4) + 4 g + j % 4,
// so W2 is staged in LDS in exactly that order, one 16-byte fragment per lane
// and (K block, column block).  LDS holds W2 (W^2 bf16), W1 fragments, b1,
// b2, W3 and b3; after staging it is read-only, and the waves run their row
// tiles without further barriers.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_bits(float x) {   // round to nearest even
  uint32_t u = __float_as_uint(x);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_val(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float silu_fast(float u) { return __fdividef(u, 1.0f + __expf(-u)); }

constexpr int kFusedMaxIn = 32, kFusedMaxOut = 4, kFusedMaxWidth = 256;

template <int W, int NO, int NS>
__global__ __launch_bounds__(NS == 2 ? 256 : 512) void mlp_fused_kernel(const float* __restrict__ P, int n_in,
                                                        int n_out, const float* __restrict__ X,
                                                        int64_t n, float* __restrict__ Y) {
  constexpr int KB = W / 32, CB = W / 16;
  __shared__ __attribute__((aligned(16))) unsigned short sW2[KB * CB * 64 * 8];
  __shared__ __attribute__((aligned(16))) unsigned short sW1[CB * 64 * 8];
  __shared__ float sB1[W], sB2[W], sW3[W * NO], sB3[NO];
  const float* W1 = P;
  const float* b1 = W1 + (int64_t)n_in * W;
  const float* W2 = b1 + W;
  const float* b2 = W2 + (int64_t)W * W;
  const float* W3 = b2 + W;
  const float* b3 = W3 + (int64_t)W * n_out;
  for (int e = threadIdx.x; e < KB * CB * 512; e += blockDim.x) {
    const int j = e & 7, ln = (e >> 3) & 63, cb = (e >> 9) % CB, kb = (e >> 9) / CB;
    const int g = ln >> 4, k = 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3), col = 16 * cb + (ln & 15);
    sW2[e] = bf16_bits(W2[k * W + col]);
  }
  for (int e = threadIdx.x; e < CB * 512; e += blockDim.x) {
    const int j = e & 7, ln = (e >> 3) & 63, c = e >> 9;
    const int i = 8 * (ln >> 4) + j, k = 16 * c + (ln & 15);
    sW1[e] = i < n_in ? bf16_bits(W1[i * W + k]) : (unsigned short)0;
  }
  for (int e = threadIdx.x; e < W; e += blockDim.x) {
    sB1[e] = b1[e];
    sB2[e] = b2[e];
    for (int o = 0; o < NO; ++o) sW3[e * NO + o] = o < n_out ? W3[e * n_out + o] : 0.0f;
  }
  if (threadIdx.x < NO) sB3[threadIdx.x] = threadIdx.x < n_out ? b3[threadIdx.x] : 0.0f;
  __syncthreads();

  const int lane = threadIdx.x & 63, g = lane >> 4, ln = lane & 15;
  const int wpb = blockDim.x >> 6;
  constexpr int RW = 16 * NS;   // rows per wave tile
  const int64_t ntiles = (n + RW - 1) / RW;
  for (int64_t t = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); t < ntiles;
       t += (int64_t)gridDim.x * wpb) {
    const int64_t r0 = t * RW;
    // layer-1 B operands: X[row][8 g + j] of rows r0 + 16 s + ln, as bf16 pairs
    bf16x8_t xh[NS], xl[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int64_t row = r0 + 16 * s + ln;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = 8 * g + j;
        const float x = (row < n && i < n_in) ? X[row * n_in + i] : 0.0f;
        const __bf16 hb = (__bf16)x;
        xh[s][j] = hb;
        xl[s][j] = (__bf16)(x - (float)hb);
      }
    }
    // layer 1 and the layer-2 A fragments (hi, lo) of both strips
    bf16x8_t ah[NS][KB], al[NS][KB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const bf16x8_t a1 = *(const bf16x8_t*)&sW1[(c * 64 + lane) * 8];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        f32x4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xl[s], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, xh[s], d, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float h = silu_fast(d[v] + sB1[16 * c + 4 * g + v]);
          const __bf16 hb = (__bf16)h;
          ah[s][c >> 1][4 * (c & 1) + v] = hb;
          al[s][c >> 1][4 * (c & 1) + v] = (__bf16)(h - (float)hb);
        }
      }
    }
    // layer 2 by column blocks, each followed by its share of layer 3
    float yp[NO][NS][4];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) yp[o][s][v] = 0.0f;
    for (int cb = 0; cb < CB; ++cb) {
      f32x4_t acc[NS][2];
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[s][0] = acc[s][1] = (f32x4_t){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const bf16x8_t b = *(const bf16x8_t*)&sW2[((kb * CB + cb) * 64 + lane) * 8];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          acc[s][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s][kb], b, acc[s][1], 0, 0, 0);
          acc[s][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s][kb], b, acc[s][0], 0, 0, 0);
        }
      }
      const int col = 16 * cb + ln;
      const float bb = sB2[col];
      float w3[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) w3[o] = sW3[col * NO + o];
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float h = silu_fast(acc[s][0][v] + acc[s][1][v] + bb);
#pragma unroll
          for (int o = 0; o < NO; ++o) yp[o][s][v] = fmaf(h, w3[o], yp[o][s][v]);
        }
    }
    // sum over the 16 lanes of each row group, then one lane per group writes
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float y = yp[o][s][v];
          y += __shfl_xor(y, 8, 64);
          y += __shfl_xor(y, 4, 64);
          y += __shfl_xor(y, 2, 64);
          y += __shfl_xor(y, 1, 64);
          yp[o][s][v] = y;
        }
    if (ln == 0) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = r0 + 16 * s + 4 * g + v;
          if (row < n)
#pragma unroll
            for (int o = 0; o < NO; ++o)
              if (o < n_out) Y[row * n_out + o] = yp[o][s][v] + sB3[o];
        }
    }
  }
}

static int grid_of(int64_t tot) {
  int64_t g = (tot + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace nm

struct nm_mlp {
  int n_in = 0, width = 0, n_out = 0;
  hipStream_t s = nullptr;
  int64_t np = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *pw = nullptr, *g = nullptr;
  int step = 0;
  int64_t cap = 0;   // batch rows the work buffers hold
  float *u1 = nullptr, *h1 = nullptr, *u2 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr,
        *du = nullptr, *xb = nullptr, *tb = nullptr;
  double *acc = nullptr, *part = nullptr;
  int64_t part_cap = 0;
  int64_t* idx = nullptr;
  std::string err;
  std::vector<void*> owned;   // parameters and optimiser state
  std::vector<void*> work;    // batch-sized buffers (replaced when a batch outgrows them)

  int64_t off_W1() const { return 0; }
  int64_t off_b1() const { return (int64_t)n_in * width; }
  int64_t off_W2() const { return off_b1() + width; }
  int64_t off_b2() const { return off_W2() + (int64_t)width * width; }
  int64_t off_W3() const { return off_b2() + width; }
  int64_t off_b3() const { return off_W3() + (int64_t)width * n_out; }
};

namespace {

void* dalloc(nm_mlp* m, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw std::string("device allocation failed");
  }
  m->owned.push_back(p);
  return p;
}

void hcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::string(what) + ": " + hipGetErrorString(e);
}

void* walloc(nm_mlp* m, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw std::string("device allocation failed");
  }
  m->work.push_back(p);
  return p;
}

void ensure(nm_mlp* m, int64_t n) {
  if (n <= m->cap) return;
  // release the old work buffers once the stream is idle
  hcheck(hipStreamSynchronize(m->s), "sync");
  for (void* q : m->work) (void)hipFree(q);
  m->work.clear();
  m->part = nullptr;
  m->part_cap = 0;
  const int w = std::max(m->width, m->n_out), wi = std::max(m->n_in, w);
  float** fb[] = {&m->u1, &m->h1, &m->u2, &m->h2, &m->du};
  for (float** q : fb) *q = (float*)walloc(m, (size_t)n * w * sizeof(float));
  m->y = (float*)walloc(m, (size_t)n * m->n_out * sizeof(float));
  m->dy = (float*)walloc(m, (size_t)n * m->n_out * sizeof(float));
  m->xb = (float*)walloc(m, (size_t)n * wi * sizeof(float));
  m->tb = (float*)walloc(m, (size_t)n * m->n_out * sizeof(float));
  m->acc = (double*)walloc(m, (size_t)n * w * sizeof(double));
  m->idx = (int64_t*)walloc(m, (size_t)n * sizeof(int64_t));
  m->cap = n;
}

// fp64 scratch for split-K partials and reductions (grown on demand; the
// old block is released only after the stream has drained)
double* partials(nm_mlp* m, int64_t len) {
  if (len > m->part_cap) {
    hcheck(hipStreamSynchronize(m->s), "sync");
    if (m->part) {
      for (auto it = m->work.begin(); it != m->work.end(); ++it)
        if (*it == (void*)m->part) { (void)hipFree(*it); m->work.erase(it); break; }
    }
    m->part = (double*)walloc(m, (size_t)len * sizeof(double));
    m->part_cap = len;
  }
  return m->part;
}

void kchk(int rc, const char* what) {
  if (rc != 0) throw std::string("kernel launch failed: ") + what;
}

// G[M][N] (fp32) = A^T B with A [K][M], B [K][N] row-major, K = batch rows:
// K split into chunks on grid.z, fp64 partials folded in order.
void grad_tn(nm_mlp* m, const float* A, int M, const float* B, int N, int64_t K, float* G) {
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(256, K / 2048));
  const int64_t kc = ((K + ns - 1) / ns + 15) / 16 * 16;
  ns = (K + kc - 1) / kc;
  const int64_t klast = K - (ns - 1) * kc;
  double* part = partials(m, ns * (int64_t)M * N);
  kchk(nm::gemm_f32acc(m->s, true, false, M, N, (int)kc, (int)ns, 1.0, A, M, kc * M, B, N, kc * N,
                       0.0, part, N, (int64_t)M * N, (int)klast),
       "weight gradient");
  hipLaunchKernelGGL(nm::fold_f32_kernel, dim3(nm::grid_of((int64_t)M * N)), dim3(256), 0, m->s,
                     part, (int)ns, (int64_t)M * N, G);
}

void colsum(nm_mlp* m, const float* x, int64_t n, int w, float* out) {
  const int64_t rpc = 4096;
  const int64_t nch = (n + rpc - 1) / rpc;
  double* part = partials(m, nch * w);
  hipLaunchKernelGGL(nm::colsum_partial_kernel, dim3((w + 63) / 64, (unsigned)nch), dim3(256), 0,
                     m->s, x, n, w, rpc, part);
  hipLaunchKernelGGL(nm::fold_f32_kernel, dim3(nm::grid_of(w)), dim3(256), 0, m->s, part,
                     (int)nch, (int64_t)w, out);
}

// forward of n rows of X with the given work buffers: acc (fp64 GEMM output,
// n x max(width, n_out)), pre-activations u1, u2 (kept for the backward pass;
// may be null) and activations h1, h2 (n x width); output y (n x n_out)
void forward_rows(nm_mlp* m, int64_t n, const float* X, double* acc, float* u1, float* h1,
                  float* u2, float* h2, float* y) {
  const int w = m->width;
  const float* P = m->pw;
  kchk(nm::gemm_f32acc(m->s, false, false, (int)n, w, m->n_in, 1, 1.0, X, m->n_in, 0,
                       P + m->off_W1(), w, 0, 0.0, acc, w, 0),
       "layer 1");
  hipLaunchKernelGGL(nm::bias_act_kernel, dim3(nm::grid_of(n * w)), dim3(256), 0, m->s, acc,
                     P + m->off_b1(), u1, h1, n, w, 1);
  kchk(nm::gemm_f32acc(m->s, false, false, (int)n, w, w, 1, 1.0, h1, w, 0, P + m->off_W2(), w,
                       0, 0.0, acc, w, 0),
       "layer 2");
  hipLaunchKernelGGL(nm::bias_act_kernel, dim3(nm::grid_of(n * w)), dim3(256), 0, m->s, acc,
                     P + m->off_b2(), u2, h2, n, w, 1);
  kchk(nm::gemm_f32acc(m->s, false, false, (int)n, m->n_out, w, 1, 1.0, h2, w, 0,
                       P + m->off_W3(), m->n_out, 0, 0.0, acc, m->n_out, 0),
       "layer 3");
  hipLaunchKernelGGL(nm::bias_act_kernel, dim3(nm::grid_of(n * m->n_out)), dim3(256), 0, m->s,
                     acc, P + m->off_b3(), (float*)nullptr, y, n, m->n_out, 0);
}

// forward of n rows of X (in the work buffers); output in m->y
void forward(nm_mlp* m, int64_t n, const float* X) {
  forward_rows(m, n, X, m->acc, m->u1, m->h1, m->u2, m->h2, m->y);
}

// loss and gradient (into m->g) of n rows (X, T device)
double loss_grad(nm_mlp* m, int64_t n, const float* X, const float* T) {
  const int w = m->width, no = m->n_out;
  forward(m, n, X);
  const int64_t cnt = n * no;
  const int nb = std::min<int64_t>(1024, (cnt + 255) / 256);
  double* part = partials(m, std::max<int64_t>(nb, 1));
  hipLaunchKernelGGL(nm::mse_kernel, dim3(nb), dim3(256), 0, m->s, m->y, T, m->dy, cnt, part);
  std::vector<double> hp(nb);
  hcheck(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, m->s), "D2H");
  hcheck(hipStreamSynchronize(m->s), "sync");
  double loss = 0.0;
  for (double x : hp) loss += x;
  loss = 0.5 * loss / (double)cnt;
  float* G = m->g;
  const float* P = m->pw;
  // layer 3
  grad_tn(m, m->h2, w, m->dy, no, n, G + m->off_W3());
  colsum(m, m->dy, n, no, G + m->off_b3());
  kchk(nm::gemm_f32acc(m->s, false, true, (int)n, w, no, 1, 1.0, m->dy, no, 0, P + m->off_W3(), no,
                       0, 0.0, m->acc, w, 0),
       "dh2");
  hipLaunchKernelGGL(nm::act_back_kernel, dim3(nm::grid_of(n * w)), dim3(256), 0, m->s, m->acc,
                     m->u2, m->du, n * w);
  // layer 2
  grad_tn(m, m->h1, w, m->du, w, n, G + m->off_W2());
  colsum(m, m->du, n, w, G + m->off_b2());
  kchk(nm::gemm_f32acc(m->s, false, true, (int)n, w, w, 1, 1.0, m->du, w, 0, P + m->off_W2(), w, 0,
                       0.0, m->acc, w, 0),
       "dh1");
  hipLaunchKernelGGL(nm::act_back_kernel, dim3(nm::grid_of(n * w)), dim3(256), 0, m->s, m->acc,
                     m->u1, m->du, n * w);
  // layer 1
  grad_tn(m, X, m->n_in, m->du, w, n, G + m->off_W1());
  colsum(m, m->du, n, w, G + m->off_b1());
  return loss;
}

// the fused inference kernel takes widths that are multiples of 32 up to 256,
// up to 32 inputs and up to 4 outputs
bool fused_fits(const nm_mlp* m) {
  return m->width % 32 == 0 && m->width <= nm::kFusedMaxWidth && m->n_in <= nm::kFusedMaxIn &&
         m->n_out <= nm::kFusedMaxOut;
}

// one 16-row strip per wave, eight waves per workgroup (two per SIMD: the
// strip's A fragments take 64 registers); measured 25 % faster than two
// strips per wave with four waves (7.5 against 9.9 ms for 17.6 M rows)
template <int W>
void launch_fused(nm_mlp* m, int64_t n, const float* X, float* Y) {
  constexpr int kStrips = 1, kWaves = 8;
  const int64_t tiles = (n + 16 * kStrips - 1) / (16 * kStrips);
  const dim3 grid((unsigned)std::min<int64_t>((tiles + kWaves - 1) / kWaves, 1024)), block(64 * kWaves);
  if (m->n_out == 1)
    hipLaunchKernelGGL((nm::mlp_fused_kernel<W, 1, kStrips>), grid, block, 0, m->s, m->pw, m->n_in,
                       m->n_out, X, n, Y);
  else
    hipLaunchKernelGGL((nm::mlp_fused_kernel<W, nm::kFusedMaxOut, kStrips>), grid, block, 0, m->s,
                       m->pw, m->n_in, m->n_out, X, n, Y);
}

// Y [n][n_out] from X [n][n_in] in one kernel (no work buffers)
void forward_fused(nm_mlp* m, int64_t n, const float* X, float* Y) {
  if (n <= 0) return;
  switch (m->width) {
    case 32: launch_fused<32>(m, n, X, Y); break;
    case 64: launch_fused<64>(m, n, X, Y); break;
    case 96: launch_fused<96>(m, n, X, Y); break;
    case 128: launch_fused<128>(m, n, X, Y); break;
    case 160: launch_fused<160>(m, n, X, Y); break;
    case 192: launch_fused<192>(m, n, X, Y); break;
    case 224: launch_fused<224>(m, n, X, Y); break;
    case 256: launch_fused<256>(m, n, X, Y); break;
    default: throw std::string("fused inference: unsupported width");
  }
  hcheck(hipGetLastError(), "fused inference");
}

int fail(nm_mlp* m, const std::string& e) {
  if (m) m->err = e;
  return CC_ERR_HIP;
}

}  // namespace

// ------------------------------------------------ allocation-free forward
// Work area of mlp_forward_noalloc: a fixed device array, so that the call
// needs no device allocation.  Each GPU the library runs on holds its own
// copy until the process ends.  In host code the array's name is only a
// stand-in: its device address, per device, comes from hipGetSymbolAddress
// (taken once per device, with that device current) and only that address
// is handed to kernels.  All calls on one GPU share that GPU's copy, which
// keeps the last call's contents; calls that overlap on one GPU (other
// streams or host threads) race on it and must be serialised by the caller.
constexpr size_t kScratchBytes = (size_t)32 << 20;   // 32 MiB
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;   // device address of scratch, by device

// scratch's device address on the device that runs stream s
void* scratch_on(hipStream_t s) {
  int dev = 0;
  if (s)
    hcheck(hipStreamGetDevice(s, &dev), "stream device");
  else
    hcheck(hipGetDevice(&dev), "current device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    int cur = 0;
    hcheck(hipGetDevice(&cur), "current device");
    if (cur != dev) hcheck(hipSetDevice(dev), "set device");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    hcheck(e, "work area address");
    if (!p) throw std::string("work area address is null");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int mlp_create(nm_mlp** out, int n_in, int width, int n_out, uint64_t seed, void* stream) {
  if (!out || n_in < 1 || width < 1 || n_out < 1 || n_in > 4096 || width > 4096 || n_out > 4096)
    return CC_ERR_ARG;
  nm_mlp* m = new nm_mlp;
  m->n_in = n_in;
  m->width = width;
  m->n_out = n_out;
  m->s = (hipStream_t)stream;
  try {
    m->np = m->off_b3() + n_out;
    m->p = (float*)dalloc(m, m->np * sizeof(float));
    m->m = (float*)dalloc(m, m->np * sizeof(float));
    m->v = (float*)dalloc(m, m->np * sizeof(float));
    m->pw = (float*)dalloc(m, m->np * sizeof(float));
    m->g = (float*)dalloc(m, m->np * sizeof(float));
    // N(0, 1/fan_in) weights, zero biases
    std::vector<float> h(m->np, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    auto fill_w = [&](int64_t off, int fin, int fout) {
      const double sc = 1.0 / std::sqrt((double)fin);
      for (int64_t k = 0; k < (int64_t)fin * fout; ++k) h[off + k] = (float)(sc * nd(rng));
    };
    fill_w(m->off_W1(), n_in, width);
    fill_w(m->off_W2(), width, width);
    fill_w(m->off_W3(), width, n_out);
    *out = m;
    return mlp_set_params(m, h.data());
  } catch (const std::string& e) {
    for (void* q : m->owned) (void)hipFree(q);
    delete m;
    *out = nullptr;
    return CC_ERR_OOM;
  }
}

int64_t mlp_num_params(const nm_mlp* m) { return m ? m->np : -1; }

int mlp_dims(const nm_mlp* m, int* n_in, int* width, int* n_out) {
  if (!m) return CC_ERR_ARG;
  if (n_in) *n_in = m->n_in;
  if (width) *width = m->width;
  if (n_out) *n_out = m->n_out;
  return CC_OK;
}

int mlp_set_params(nm_mlp* m, const float* src) {
  if (!m || !src) return CC_ERR_ARG;
  try {
    hcheck(hipMemcpyAsync(m->p, src, m->np * sizeof(float), hipMemcpyHostToDevice, m->s), "H2D");
    hcheck(hipMemsetAsync(m->m, 0, m->np * sizeof(float), m->s), "memset");
    hcheck(hipMemsetAsync(m->v, 0, m->np * sizeof(float), m->s), "memset");
    hipLaunchKernelGGL(nm::round_kernel, dim3(nm::grid_of(m->np)), dim3(256), 0, m->s, m->p, m->pw,
                       m->np);
    hcheck(hipGetLastError(), "round");
    hcheck(hipStreamSynchronize(m->s), "sync");
    m->step = 0;
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_get_params(nm_mlp* m, float* dst, int working) {
  if (!m || !dst) return CC_ERR_ARG;
  try {
    hcheck(hipMemcpyAsync(dst, working ? m->pw : m->p, m->np * sizeof(float), hipMemcpyDeviceToHost,
                          m->s),
           "D2H");
    hcheck(hipStreamSynchronize(m->s), "sync");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_forward(nm_mlp* m, int64_t n, const float* X, float* Y) {
  if (!m || n < 0 || (n > 0 && (!X || !Y))) return CC_ERR_ARG;
  try {
    if (fused_fits(m)) {
      forward_fused(m, n, X, Y);
      hcheck(hipStreamSynchronize(m->s), "sync");
      return CC_OK;
    }
    const int64_t chunk = 1 << 20;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
      const int64_t k = std::min(chunk, n - r0);
      ensure(m, k);
      forward(m, k, X + r0 * m->n_in);
      hcheck(hipMemcpyAsync(Y + r0 * m->n_out, m->y, k * m->n_out * sizeof(float),
                            hipMemcpyDeviceToDevice, m->s),
             "D2D");
    }
    hcheck(hipGetLastError(), "forward");
    hcheck(hipStreamSynchronize(m->s), "sync");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_forward_noalloc(nm_mlp* m, int64_t n, const float* X, float* Y) {
  if (!m || n < 0 || (n > 0 && (!X || !Y))) return CC_ERR_ARG;
  // per row: one fp64 GEMM output row and the two hidden activations (fp32);
  // rows go through the work area in chunks of a multiple of 64
  const int w = m->width, wa = std::max(m->width, m->n_out);
  const size_t per_row = (size_t)wa * sizeof(double) + 2 * (size_t)w * sizeof(float);
  int64_t rows = (int64_t)((kScratchBytes - 3 * 256) / per_row) / 64 * 64;
  if (rows < 64) {
    m->err = "network too wide for the work area of mlp_forward_noalloc (" +
             std::to_string(kScratchBytes) + " bytes, 64 rows at a time)";
    return CC_ERR_ARG;
  }
  try {
    if (n == 0) return CC_OK;
    if (fused_fits(m)) {   // the fused kernel needs no work area
      forward_fused(m, n, X, Y);
      hcheck(hipStreamSynchronize(m->s), "sync");
      return CC_OK;
    }
    char* base = (char*)scratch_on(m->s);
    double* acc = (double*)base;
    float* h1 = (float*)(base + align256((size_t)rows * wa * sizeof(double)));
    float* h2 = (float*)((char*)h1 + align256((size_t)rows * w * sizeof(float)));
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
      const int64_t k = std::min(rows, n - r0);
      forward_rows(m, k, X + r0 * m->n_in, acc, nullptr, h1, nullptr, h2, Y + r0 * m->n_out);
    }
    hcheck(hipGetLastError(), "forward");
    hcheck(hipStreamSynchronize(m->s), "sync");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_loss_grad(nm_mlp* m, int64_t n, const float* X, const float* T, double* loss, float* grad) {
  if (!m || n < 1 || !X || !T) return CC_ERR_ARG;
  try {
    ensure(m, n);
    const double l = loss_grad(m, n, X, T);
    if (loss) *loss = l;
    if (grad) {
      hcheck(hipMemcpyAsync(grad, m->g, m->np * sizeof(float), hipMemcpyDeviceToHost, m->s), "D2H");
    }
    hcheck(hipGetLastError(), "loss_grad");
    hcheck(hipStreamSynchronize(m->s), "sync");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_adam_step(nm_mlp* m, float lr) {
  if (!m || !(lr > 0)) return CC_ERR_ARG;
  try {
    ++m->step;
    const float c1 = 1.0f - std::pow(0.9f, (float)m->step);
    const float c2 = 1.0f - std::pow(0.999f, (float)m->step);
    hipLaunchKernelGGL(nm::adam_kernel, dim3(nm::grid_of(m->np)), dim3(256), 0, m->s, m->p, m->m,
                       m->v, m->g, m->pw, m->np, lr, c1, c2);
    hcheck(hipGetLastError(), "adam");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

int mlp_train(nm_mlp* m, int64_t n, const float* X, const float* T, int64_t batch, int steps,
              float lr, uint64_t seed, double* last_loss) {
  if (!m || n < 1 || !X || !T || batch < 1 || steps < 0 || !(lr > 0)) return CC_ERR_ARG;
  try {
    batch = std::min(batch, n);
    ensure(m, batch);
    std::mt19937_64 rng(seed);
    std::uniform_int_distribution<int64_t> pick(0, n - 1);
    std::vector<int64_t> hidx(batch);
    double l = 0.0;
    for (int s = 0; s < steps; ++s) {
      for (auto& q : hidx) q = pick(rng);
      hcheck(hipMemcpyAsync(m->idx, hidx.data(), batch * sizeof(int64_t), hipMemcpyHostToDevice,
                            m->s),
             "H2D");
      hipLaunchKernelGGL(nm::gather_rows_kernel, dim3(nm::grid_of(batch * m->n_in)), dim3(256), 0,
                         m->s, X, m->idx, batch, m->n_in, m->xb);
      hipLaunchKernelGGL(nm::gather_rows_kernel, dim3(nm::grid_of(batch * m->n_out)), dim3(256), 0,
                         m->s, T, m->idx, batch, m->n_out, m->tb);
      l = loss_grad(m, batch, m->xb, m->tb);
      const int rc = mlp_adam_step(m, lr);
      if (rc != CC_OK) return rc;
    }
    if (last_loss) *last_loss = l;
    hcheck(hipStreamSynchronize(m->s), "sync");
    return CC_OK;
  } catch (const std::string& e) {
    return fail(m, e);
  }
}

const char* mlp_last_error(const nm_mlp* m) { return m ? m->err.c_str() : "null network"; }

void mlp_destroy(nm_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->s);
  for (void* q : m->work) (void)hipFree(q);
  for (void* q : m->owned) (void)hipFree(q);
  delete m;
}

}  // extern "C"
