// Host-side launchers of the device kernels (see kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace nm {

constexpr int kMaxViewDims = 6;
constexpr int kMaxRows = 128;   // subspace rows handled by rows_dot / rows_axpy
constexpr int kMaxRhs = 4;      // right-hand sides of rows_dot_multi / rows_axpy_multi

// A strided map between an output box and an input tensor:
// out[obase + sum_d i_d ostr_d]  <->  in[ibase + sum_d i_d istr_d + sum_r j_r rstr_r]
// for 0 <= i_d < dims[d] and 0 <= j_r < rdims[r] (j_r are summed over).
struct ViewSpec {
  int nd = 0;
  int nr = 0;
  int64_t obase = 0, ibase = 0;
  int64_t dims[kMaxViewDims] = {0};
  int64_t ostr[kMaxViewDims] = {0};
  int64_t istr[kMaxViewDims] = {0};
  int64_t rdims[2] = {0, 0};
  int64_t rstr[2] = {0, 0};
};

int gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, int batch, double alpha,
             const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb,
             int64_t sB, double beta, double* C, int64_t ldc, int64_t sC, int Klast = 0);
int view_gather(hipStream_t s, double* out, const double* in, const ViewSpec& v, double alpha,
                double beta);
int view_gather_f32(hipStream_t s, float* out, const double* in, const ViewSpec& v);
// BF16 split-precision GEMM: C = alpha A B + beta C with A [M][K] and B^T [N][K]
// given as bfloat16 pairs (hi, lo) in uint16 storage; K and Klast multiples
// of 32, lda / ldb / batch strides multiples of 8, 16-byte aligned pointers.
// tile: 0 = 128 x 128 outputs per workgroup (two per CU), 1 = 256 x 256,
// 2 = 256 x 128, 3 = 128 x 256 (one per CU), 4 = 256 x 128 and 5 = 128 x 256
// with loads two K steps ahead, 6 = 256 x 128 and 7 = 128 x 256 with the next
// step's fragments read during this step's products; -1 =
// bf16x3_auto_tile's choice.
constexpr int kBf16Tiles = 8;
int bf16x3_auto_tile(int M, int N, int batch);
void bf16x3_tile_dims(int tile, int& bm, int& bn);
// A, B: interleaved bfloat16 pair arrays (element k of a row: hi at
// 2 (k - k % 8) + k % 8, lo 8 further); lda, ldb, sA, sB in uint16 units
// (lda, ldb >= 2 K); a K offset k0 along a row is 2 k0 elements
int gemm_bf16x3(hipStream_t s, int M, int N, int K, int batch, double alpha, const uint16_t* A,
                int64_t lda, int64_t sA, const uint16_t* B, int64_t ldb, int64_t sB, double beta,
                double* C, int64_t ldc, int64_t sC, int Klast, int tile = -1);
// bfloat16 pairs of a strided double view whose output strides address a
// [rows][Kp] plane, written interleaved into out ([rows][2 Kp] uint16);
// padding [K, Kp) zeroed
int view_gather_bf16x2(hipStream_t s, uint16_t* out, const double* in, const ViewSpec& v, int64_t rows,
                       int K, int Kp);
int gemm_f32acc(hipStream_t s, bool ta, bool tb, int M, int N, int K, int batch, double alpha,
                const float* A, int64_t lda, int64_t sA, const float* B, int64_t ldb, int64_t sB,
                double beta, double* C, int64_t ldc, int64_t sC, int Klast = 0);
int view_scatter(hipStream_t s, double* in, const double* out, const ViewSpec& v, double alpha);
int fill(hipStream_t s, double* x, double val, int64_t n);
int axpby(hipStream_t s, double* y, const double* x, double a, double b, int64_t n);
// rows of len doubles: dst[r ldd + j] = src[r lds + j]
int rows_copy(hipStream_t s, double* dst, int64_t ldd, const double* src, int64_t lds, int64_t len,
              int64_t rows);
int apply_denominator(hipStream_t s, double* y, const double* x, const double* eps, int o, int v,
                      double shift, int mode);
int apply_metric(hipStream_t s, double* y, const double* x, int o, int v, int mode);
// Half layout of amplitude-shaped vectors: singles, then the doubles of the
// unordered pairs (ia) <= (jb) (o v + o v (o v + 1) / 2 doubles), in which the
// biorthonormal product of symmetric vectors is the plain dot product.
int half_pack(hipStream_t s, double* h, const double* x, int o, int v);
int half_unpack(hipStream_t s, double* x, const double* h, int o, int v);
// y = x / (shift - D) on the half layout (the Davidson preconditioner)
int half_denominator(hipStream_t s, double* y, const double* x, const double* eps, int o, int v,
                     double shift);
int dot(hipStream_t s, const double* x, const double* y, int64_t n, int o, int v, int packed,
        double* scratch, double* out_dev);
int absmax(hipStream_t s, const double* x, int64_t n, double* scratch, double* out_dev);
int reduce_scratch_doubles();
int rows_dot(hipStream_t s, const double* V, int m, int64_t n, const double* x, double* part,
             double* out);
int rows_scratch_doubles();
// out[r][k] = <V_k, X_r> for R <= kMaxRhs vectors X_r = X + r ldx (device out)
int rows_dot_multi(hipStream_t s, const double* V, int m, int64_t n, const double* X, int64_t ldx,
                   int R, double* part, double* out);
// X_r += alpha sum_k H[r][k] V_k (H device [R][m]); overwrite: X_r = alpha sum ...
int rows_axpy_multi(hipStream_t s, const double* V, int m, int64_t n, const double* H, double alpha,
                    double* X, int64_t ldx, int R, bool overwrite = false);
int rows_axpy(hipStream_t s, const double* V, int m, int64_t n, const double* h, double alpha,
              double* x);

// Blocked two-electron density (density.hip).
// Symmetric index pairs of an n x n matrix (n = o + v) in the order
// [oo (p >= q) | ov (k, c) | vv (a >= c)], m = n (n + 1) / 2 of them:
// out[r][j] = in[r][p][q] + in[r][q][p] (sum, p != q) or in[r][p][q] (p >= q).
int pack_pairs(hipStream_t s, double* out, int64_t ldo, const double* in, int64_t ldi, int64_t rows,
               int o, int v, bool sum);
// Rows (a >= c) with c in [c0, c0 + cc) of out[(a >= c)][(b >= d)] (pairs
// packed as x (x + 1) / 2 + y) = the sum over the distinct images
// (a, c) <-> (c, a), (b, d) <-> (d, b) of G[c][d][a][b], from the chunk's two
// images M1c[c - c0][d][a][b] = G[c][d][a][b] ([cc][v][v][v]) and
// M2c[a][d][c - c0][b] = G[a][d][c][b] ([v][v][cc][v]).
int pack_vvvv_rows(hipStream_t s, double* out, const double* M1c, const double* M2c, int v, int c0,
                   int cc);
// out[r] = alpha sum_j A[r lda + j] B[r ldb + j] + beta out[r]  (j < len; ldb 0
// broadcasts one row of B)
int rowdot(hipStream_t s, double* out, const double* A, int64_t lda, const double* B, int64_t ldb,
           int64_t rows, int64_t len, double alpha, double beta);

}  // namespace nm
