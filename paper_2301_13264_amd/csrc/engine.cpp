// Device tensor engine with a recording tape (see engine.h).
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <set>

namespace nm {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    throw Error(-3, std::string(what) + ": " + hipGetErrorString(e));
}

static void kcheck(int rc, const char* what) {
  if (rc != 0) throw Error(-3, std::string("kernel launch failed: ") + what);
}

// ------------------------------------------------------------------- Arena
Arena::~Arena() {
  for (auto& c : chunks_) (void)hipFree(c.base);
}

double* Arena::alloc(int64_t ndouble) {
  size_t bytes = ((size_t)std::max<int64_t>(ndouble, 1) * sizeof(double) + 255) & ~size_t(255);
  while (true) {
    if (cur_ < chunks_.size()) {
      Chunk& c = chunks_[cur_];
      if (c.top + bytes <= c.cap) {
        double* p = (double*)(c.base + c.top);
        c.top += bytes;
        live_ += bytes;
        peak_ = std::max(peak_, live_);
        return p;
      }
      // chunks after the current one are unused: take the first that fits
      for (size_t k = cur_ + 1; k < chunks_.size(); ++k) {
        if (chunks_[k].cap >= bytes) {
          std::swap(chunks_[cur_ + 1], chunks_[k]);
          ++cur_;
          chunks_[cur_].top = 0;
          break;
        }
      }
      if (chunks_[cur_].top + bytes <= chunks_[cur_].cap) continue;
      // none fits: release the unused ones (after the device has finished
      // with whatever they held) so that capacity is not stranded
      if (cur_ + 1 < chunks_.size()) {
        (void)hipDeviceSynchronize();
        for (size_t k = cur_ + 1; k < chunks_.size(); ++k) (void)hipFree(chunks_[k].base);
        chunks_.resize(cur_ + 1);
      }
    }
    size_t cap = std::max(bytes, (size_t)1 << 30);
    char* base = nullptr;
    if (std::getenv("NACME_VERBOSE"))
      std::fprintf(stderr, "[arena] new chunk %.3f GB (%zu held)\n", cap / 1e9, chunks_.size());
    hipError_t e = hipMalloc(&base, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(-4, "device allocation of " + std::to_string(cap) + " bytes failed");
    }
    chunks_.push_back({base, cap, 0});
    cur_ = chunks_.size() - 1;
  }
}

void Arena::trim() {
  if (cur_ + 1 >= chunks_.size()) return;
  (void)hipDeviceSynchronize();
  for (size_t k = cur_ + 1; k < chunks_.size(); ++k) (void)hipFree(chunks_[k].base);
  chunks_.resize(cur_ + 1);
}

void Arena::rewind(Mark m) {
  if (chunks_.empty()) return;
  // recompute live bytes: chunks before m.chunk full up to their top
  for (size_t k = m.chunk + 1; k < chunks_.size(); ++k) chunks_[k].top = 0;
  cur_ = m.chunk;
  chunks_[cur_].top = m.top;
  size_t live = 0;
  for (size_t k = 0; k <= cur_; ++k) live += chunks_[k].top;
  live_ = live;
}

size_t Arena::reserved_bytes() const {
  size_t s = 0;
  for (auto& c : chunks_) s += c.cap;
  return s;
}

// ------------------------------------------------------------------ helpers
Tensor make_tensor(Arena& a, const std::vector<int64_t>& shape, bool zero, hipStream_t s) {
  Tensor t;
  t.nd = (int)shape.size();
  if (t.nd > kMaxViewDims) throw Error(-1, "tensor rank too large");
  for (int k = 0; k < t.nd; ++k) t.d[k] = shape[k];
  t.p = a.alloc(t.size());
  if (zero) kcheck(fill(s, t.p, 0.0, t.size()), "fill");
  return t;
}

static void strides_of(const Tensor& t, int64_t* st) {
  int64_t s = 1;
  for (int k = t.nd - 1; k >= 0; --k) {
    st[k] = s;
    s *= t.d[k];
  }
}

DView full_view(const Tensor& t, const std::string& lab) {
  if ((int)lab.size() != t.nd) throw Error(-1, "label count mismatch");
  DView v;
  v.p = t.p;
  v.nd = t.nd;
  v.constant = t.constant;
  v.frozen = t.frozen;
  strides_of(t, v.str);
  for (int k = 0; k < t.nd; ++k) {
    v.dims[k] = t.d[k];
    v.lab[k] = lab[k];
  }
  return v;
}

static int find_lab(const DView& v, char c) {
  for (int k = 0; k < v.nd; ++k)
    if (v.lab[k] == c) return k;
  return -1;
}

// Is `v` a contiguous row-major tensor when its dims are taken in label
// order `order`?
static bool contiguous_in(const DView& v, const std::string& order) {
  int64_t s = 1;
  for (int k = (int)order.size() - 1; k >= 0; --k) {
    const int d = find_lab(v, order[k]);
    if (d < 0) return false;
    if (v.dims[d] != 1 && v.str[d] != s) return false;
    s *= v.dims[d];
  }
  return true;
}

static bool trace_on() { return std::getenv("NACME_TRACE") != nullptr; }

// NACME_TRACE: every contraction and linear term is timed on its own (stream
// synchronised before and after) and printed to stderr with its labels and
// extents, so that the cost of each term of a graph can be read off.
struct TermTrace {
  hipStream_t s;
  bool on;
  std::string what;
  std::chrono::steady_clock::time_point t0;
  static std::string desc(const DView& v) {
    std::string r(v.lab, v.lab + v.nd);
    r += "(";
    for (int k = 0; k < v.nd; ++k) r += (k ? "," : "") + std::to_string(v.dims[k]);
    return r + ")";
  }
  TermTrace(hipStream_t st, const char* kind, const DView& a, const DView* b, const DView& c)
      : s(st), on(trace_on()) {
    if (!on) return;
    what = std::string(kind) + " " + desc(a) + (b ? " " + desc(*b) : "") + " -> " + desc(c);
    (void)hipStreamSynchronize(s);
    t0 = std::chrono::steady_clock::now();
  }
  ~TermTrace() {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[term] %s %.4f ms\n", what.c_str(), ms);
  }
};

// ------------------------------------------------------------------ Engine
Engine::~Engine() {
  for (auto& kv : f32_cache_) (void)hipFree(kv.second);
  for (auto& kv : bf16_cache_) (void)hipFree(kv.second);
  clear_frozen();
}

// Packings of frozen views: up to 8 GB, each entry its own allocation so
// that the arena's LIFO order is untouched; freed once the stream has drained.
void Engine::clear_frozen() {
  if (frozen_cache_.empty()) return;
  (void)hipStreamSynchronize(s_);
  for (auto& kv : frozen_cache_) (void)hipFree(kv.second);
  frozen_cache_.clear();
  frozen_cache_bytes_ = 0;
}

void* Engine::frozen_lookup(const std::string& key) const {
  auto it = frozen_cache_.find(key);
  return it == frozen_cache_.end() ? nullptr : it->second;
}

void* Engine::frozen_store(const std::string& key, size_t bytes) {
  if (frozen_cache_bytes_ + bytes > ((size_t)8 << 30)) return nullptr;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  frozen_cache_[key] = p;
  frozen_cache_bytes_ += bytes;
  return p;
}

Engine::Engine(hipStream_t s) : s_(s) {
  red_ = arena_.alloc(reduce_scratch_doubles());
  scal_ = arena_.alloc(64);
}

double* Engine::scratch_reduce() { return red_; }
double* Engine::scalar_slot(int k) { return scal_ + k; }

// dst (+)= alpha * sum over labels of src not in dst of src, dst labels in src.
static bool same_compact(const DView& a, const DView& b) {
  if (a.nd != b.nd) return false;
  int64_t s = 1;
  for (int k = a.nd - 1; k >= 0; --k) {
    if (a.lab[k] != b.lab[k] || a.dims[k] != b.dims[k]) return false;
    if (a.dims[k] != 1 && (a.str[k] != s || b.str[k] != s)) return false;
    s *= a.dims[k];
  }
  return true;
}

static void gather_into(hipStream_t s, double alpha, const DView& src, const DView& dst,
                        double beta) {
  if (src.nd > 0 && same_compact(src, dst)) {
    int64_t n = 1;
    for (int k = 0; k < src.nd; ++k) n *= src.dims[k];
    kcheck(axpby(s, dst.p, src.p, alpha, beta, n), "axpby");
    return;
  }
  ViewSpec vs;
  vs.nd = dst.nd;
  vs.obase = 0;
  vs.ibase = 0;
  for (int k = 0; k < dst.nd; ++k) {
    const int j = find_lab(src, dst.lab[k]);
    if (j < 0) throw Error(-1, std::string("label '") + dst.lab[k] + "' missing in source");
    if (src.dims[j] != dst.dims[k]) throw Error(-1, "dimension mismatch in view copy");
    vs.dims[k] = dst.dims[k];
    vs.ostr[k] = dst.str[k];
    vs.istr[k] = src.str[j];
  }
  for (int j = 0; j < src.nd; ++j) {
    if (find_lab(dst, src.lab[j]) >= 0) continue;
    if (vs.nr == 2) throw Error(-1, "more than two summed labels in a view term");
    vs.rdims[vs.nr] = src.dims[j];
    vs.rstr[vs.nr] = src.str[j];
    vs.nr++;
  }
  if (vs.nd == 0) {  // scalar output: treat as one element
    vs.nd = 1;
    vs.dims[0] = 1;
    vs.ostr[0] = 0;
    vs.istr[0] = 0;
  }
  // kernel indexes relative to pointers; pass them via base pointer args
  kcheck(view_gather(s, dst.p, src.p, vs, alpha, beta), "view_gather");
}

// dst (labels ld) += alpha * broadcast(src (labels ls)), ls subset of ld.
static void scatter_into(hipStream_t s, double alpha, const DView& src, const DView& dst) {
  ViewSpec vs;
  vs.nd = src.nd;
  for (int k = 0; k < src.nd; ++k) {
    const int j = find_lab(dst, src.lab[k]);
    if (j < 0) throw Error(-1, "broadcast target lacks a source label");
    vs.dims[k] = src.dims[k];
    vs.ostr[k] = src.str[k];
    vs.istr[k] = dst.str[j];
  }
  for (int j = 0; j < dst.nd; ++j) {
    if (find_lab(src, dst.lab[j]) >= 0) continue;
    if (vs.nr == 2) throw Error(-1, "more than two broadcast labels");
    vs.rdims[vs.nr] = dst.dims[j];
    vs.rstr[vs.nr] = dst.str[j];
    vs.nr++;
  }
  if (vs.nd == 0) {
    vs.nd = 1;
    vs.dims[0] = 1;
  }
  kcheck(view_scatter(s, dst.p, src.p, vs, alpha), "view_scatter");
}

void Engine::linear(double alpha, const DView& A, const DView& C, bool overwrite) {
  TermTrace trace(s_, "lin", A, nullptr, C);
  // forward reduction if every C label is in A, else broadcast
  bool all_in = true;
  for (int k = 0; k < C.nd; ++k)
    if (find_lab(A, C.lab[k]) < 0) all_in = false;
  if (all_in) {
    gather_into(s_, alpha, A, C, overwrite ? 0.0 : 1.0);
  } else {
    if (overwrite) throw Error(-1, "broadcast term cannot overwrite");
    scatter_into(s_, alpha, A, C);
  }
}

static DView packed_view(Arena& ar, const DView& src, const std::string& order, hipStream_t s) {
  DView d;
  d.nd = (int)order.size();
  int64_t st = 1;
  for (int k = d.nd - 1; k >= 0; --k) {
    const int j = find_lab(src, order[k]);
    d.lab[k] = order[k];
    d.dims[k] = src.dims[j];
    d.str[k] = st;
    st *= d.dims[k];
  }
  d.p = ar.alloc(st);
  gather_into(s, 1.0, src, d, 0.0);
  return d;
}

// C = alpha sum_z part[z] + beta C, the partial products summed in split
// order; the loads of four splits (and the old C) are issued together
__global__ void splitk_fold_kernel(double* C, int64_t ldc, const double* part, int M, int N,
                                   int nsplit, double alpha, double beta) {
  const int64_t tot = (int64_t)M * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / N, n = e - m * N;
    double* c = C + m * ldc + n;
    const double old = beta == 0.0 ? 0.0 : *c;
    double acc = 0.0;
    int z = 0;
    for (; z + 4 <= nsplit; z += 4) {
      const double p0 = part[(int64_t)z * tot + e], p1 = part[(int64_t)(z + 1) * tot + e];
      const double p2 = part[(int64_t)(z + 2) * tot + e], p3 = part[(int64_t)(z + 3) * tot + e];
      acc += p0;
      acc += p1;
      acc += p2;
      acc += p3;
    }
    for (; z < nsplit; ++z) acc += part[(int64_t)z * tot + e];
    *c = alpha * acc + (beta == 0.0 ? 0.0 : beta * old);
  }
}

// ---------------------------------------------- short contracted range
// C[x, f] = alpha sum_k X[x, k] F[f, k] (+ beta C): x the labels X shares
// with C, f the labels F shares with C, k the contracted labels (K < 64), F
// small; every label any stride.  Such products (a large tensor times a
// small matrix over an occupied index) are bound by memory: X is read once,
// each output written once, F sits in LDS.  Two layouts of the work:
//   x-fast: one x index per thread (C's unit-stride label is an x label),
//           X[x, :] in registers, a loop over f;
//   f-fast: one f index per lane (C's unit-stride label is an f label), a
//           loop over x indices whose X[x, :] every lane reads alike.
constexpr int kSmallKMax = 64, kSmallKF = 4096;   // K, NF * K limits (LDS: 8 (NF K + NF + K) bytes)
struct SmallK {
  int nx = 0, nk = 0, nf = 0;
  int64_t xd[kMaxViewDims], xsX[kMaxViewDims], xsC[kMaxViewDims];
  int64_t kd[kMaxViewDims], ksX[kMaxViewDims], ksF[kMaxViewDims];
  int64_t fd[kMaxViewDims], fsF[kMaxViewDims], fsC[kMaxViewDims];
  int64_t NX = 0;
  int K = 0, NF = 0;
};

__device__ inline void smallk_decode(int64_t e, int n, const int64_t* d, const int64_t* s1,
                                     const int64_t* s2, int64_t& o1, int64_t& o2) {
  o1 = 0;
  o2 = 0;
  for (int q = n - 1; q >= 0; --q) {
    const int64_t i = e % d[q];
    e /= d[q];
    o1 += i * s1[q];
    o2 += i * s2[q];
  }
}

// F into LDS ([f][k] or [k][f]) and the per-k offsets of X, per-f offsets of C
__device__ inline void smallk_stage(const double* __restrict__ F, const SmallK& sp, bool fk,
                                    double* sF, int64_t* sxk, int64_t* scf) {
  for (int e = threadIdx.x; e < sp.NF * sp.K; e += blockDim.x) {
    const int f = e / sp.K, k = e - f * sp.K;
    int64_t of, dummy, ok, okx;
    smallk_decode(f, sp.nf, sp.fd, sp.fsF, sp.fsC, of, dummy);
    smallk_decode(k, sp.nk, sp.kd, sp.ksF, sp.ksX, ok, okx);
    sF[fk ? e : k * sp.NF + f] = F[of + ok];
  }
  for (int k = threadIdx.x; k < sp.K; k += blockDim.x) {
    int64_t ok, okx;
    smallk_decode(k, sp.nk, sp.kd, sp.ksF, sp.ksX, ok, okx);
    sxk[k] = okx;
  }
  for (int f = threadIdx.x; f < sp.NF; f += blockDim.x) {
    int64_t of, oc;
    smallk_decode(f, sp.nf, sp.fd, sp.fsF, sp.fsC, of, oc);
    scf[f] = oc;
  }
  __syncthreads();
}

template <int KM>
__global__ __launch_bounds__(256) void smallk_xfast_kernel(double* __restrict__ C,
                                                           const double* __restrict__ X,
                                                           const double* __restrict__ F, SmallK sp,
                                                           double alpha, double beta) {
  extern __shared__ double smallk_lds[];   // sF [NF][K], sxk [K], scf [NF]
  double* sF = smallk_lds;
  int64_t* sxk = (int64_t*)(sF + sp.NF * sp.K);
  int64_t* scf = sxk + sp.K;
  smallk_stage(F, sp, true, sF, sxk, scf);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < sp.NX;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t ox, oc;
    smallk_decode(e, sp.nx, sp.xd, sp.xsX, sp.xsC, ox, oc);
    double xv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) xv[k] = k < sp.K ? X[ox + sxk[k]] : 0.0;
    // four outputs at a time, their old values loaded together
    int f = 0;
    for (; f + 4 <= sp.NF; f += 4) {
      double old[4], acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) old[u] = beta == 0.0 ? 0.0 : C[oc + scf[f + u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double* fr = sF + (f + u) * sp.K;
        acc[u] = 0.0;
#pragma unroll
        for (int k = 0; k < KM; ++k)
          if (k < sp.K) acc[u] = fma(xv[k], fr[k], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) C[oc + scf[f + u]] = alpha * acc[u] + (beta == 0.0 ? 0.0 : beta * old[u]);
    }
    for (; f < sp.NF; ++f) {
      const double* fr = sF + f * sp.K;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (k < sp.K) acc = fma(xv[k], fr[k], acc);
      double* c = C + oc + scf[f];
      *c = alpha * acc + (beta == 0.0 ? 0.0 : beta * (*c));
    }
  }
}

// blockIdx.y: chunk of 64 f indices; blockIdx.x strides over x indices, one
// wave per x index at a time (4 waves per workgroup)
template <int KM>
__global__ __launch_bounds__(256) void smallk_ffast_kernel(double* __restrict__ C,
                                                           const double* __restrict__ X,
                                                           const double* __restrict__ F, SmallK sp,
                                                           double alpha, double beta) {
  extern __shared__ double smallk_lds[];   // sF [K][NF], sxk [K], scf [NF]
  double* sF = smallk_lds;
  int64_t* sxk = (int64_t*)(sF + sp.NF * sp.K);
  int64_t* scf = sxk + sp.K;
  smallk_stage(F, sp, false, sF, sxk, scf);
  const int f = blockIdx.y * 64 + (threadIdx.x & 63);
  const bool fin = f < sp.NF;
  const int64_t cf = fin ? scf[f] : 0;
  for (int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); e < sp.NX; e += (int64_t)gridDim.x * 4) {
    int64_t ox, oc;
    smallk_decode(e, sp.nx, sp.xd, sp.xsX, sp.xsC, ox, oc);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < sp.K) acc = fma(X[ox + sxk[k]], fin ? sF[k * sp.NF + f] : 0.0, acc);
    if (fin) {
      double* c = C + oc + cf;
      *c = alpha * acc + (beta == 0.0 ? 0.0 : beta * (*c));
    }
  }
}

// C (+)= alpha sum_k X F over the labels of X not in C (K < 64); false when
// the sizes do not fit the short-K kernels (the caller then takes a GEMM path)
static bool smallk_contract(hipStream_t s, double alpha, const DView& X, const DView& F, const DView& C,
                            bool overwrite) {
  SmallK sp;
  int64_t K = 1, NX = 1, NF = 1;
  struct Lab { int64_t d, s1, s2, s3; };
  std::vector<Lab> xl, fl;
  for (int q = 0; q < X.nd; ++q) {
    const int jc = find_lab(C, X.lab[q]);
    if (jc < 0) {
      const int jf = find_lab(F, X.lab[q]);
      if (jf < 0 || sp.nk >= kMaxViewDims) return false;
      sp.kd[sp.nk] = X.dims[q];
      sp.ksX[sp.nk] = X.str[q];
      sp.ksF[sp.nk] = F.str[jf];
      ++sp.nk;
      K *= X.dims[q];
    } else {
      if (find_lab(F, X.lab[q]) >= 0) return false;   // batch label
      xl.push_back({X.dims[q], X.str[q], C.str[jc], 0});
      NX *= X.dims[q];
    }
  }
  for (int q = 0; q < F.nd; ++q) {
    const int jc = find_lab(C, F.lab[q]);
    if (jc >= 0) {
      fl.push_back({F.dims[q], F.str[q], C.str[jc], 0});
      NF *= F.dims[q];
    } else if (find_lab(X, F.lab[q]) < 0) {
      return false;
    }
  }
  if (K < 1 || K > kSmallKMax || NF * K > kSmallKF || NF > 2048 || NX < 1 ||
      (int)xl.size() > kMaxViewDims || (int)fl.size() > kMaxViewDims)
    return false;
  // outermost first: decreasing stride in C
  auto by_c = [](const Lab& a, const Lab& b) { return a.s2 > b.s2; };
  std::sort(xl.begin(), xl.end(), by_c);
  std::sort(fl.begin(), fl.end(), by_c);
  sp.nx = (int)xl.size();
  for (int q = 0; q < sp.nx; ++q) {
    sp.xd[q] = xl[q].d;
    sp.xsX[q] = xl[q].s1;
    sp.xsC[q] = xl[q].s2;
  }
  sp.nf = (int)fl.size();
  for (int q = 0; q < sp.nf; ++q) {
    sp.fd[q] = fl[q].d;
    sp.fsF[q] = fl[q].s1;
    sp.fsC[q] = fl[q].s2;
  }
  sp.NX = NX;
  sp.K = (int)K;
  sp.NF = (int)NF;
  // the unit-stride label of C decides which index the lanes run along
  const int64_t xmin = xl.empty() ? INT64_MAX : xl.back().s2;
  const int64_t fmin = fl.empty() ? INT64_MAX : fl.back().s2;
  const bool ffast = fmin < xmin && NF >= 16;
  const size_t lds = sizeof(double) * (size_t)(NF * K + K + NF);
  const double beta = overwrite ? 0.0 : 1.0;
#define NM_SMALLK(KERN, KM, GRID)                                                         \
  hipLaunchKernelGGL((KERN<KM>), GRID, dim3(256), lds, s, C.p, X.p, F.p, sp, alpha, beta)
#define NM_SMALLK_K(KERN, GRID)             \
  if (K <= 16) NM_SMALLK(KERN, 16, GRID);   \
  else if (K <= 32) NM_SMALLK(KERN, 32, GRID); \
  else NM_SMALLK(KERN, 64, GRID)
  if (ffast) {
    const dim3 grid((unsigned)std::min<int64_t>((NX + 3) / 4, 4096), (unsigned)((NF + 63) / 64));
    NM_SMALLK_K(smallk_ffast_kernel, grid);
  } else {
    const dim3 grid((unsigned)std::min<int64_t>((NX + 255) / 256, 8192));
    NM_SMALLK_K(smallk_xfast_kernel, grid);
  }
#undef NM_SMALLK_K
#undef NM_SMALLK
  kcheck(hipGetLastError() == hipSuccess ? 0 : -3, "short-K product");
  return true;
}

// K split of a single large-tile GEMM.  A workgroup of 128 x 128 output
// takes about `us_per_k` microseconds per unit of K when the device is full
// and 512 workgroups (two per CU) run at once, so a grid of `tiles`
// workgroups finishes in ceil(tiles / 512) rounds; splitting K into ns chunks
// trades rounds against chunk length plus the fold of ns partial products
// (16 bytes per element and chunk at about 4 TB/s).
constexpr double kF64UsPerK = 0.23, kF32UsPerK = 0.13, kBF16UsPerK = 0.06;
static int64_t big_split(int64_t tiles, int64_t K, int64_t MN, double us_per_k, int64_t conc = 512) {
  int64_t best = 1;
  double tbest = 1e300;
  for (int64_t ns = 1; ns <= 256; ++ns) {
    const int64_t kc = ((K + ns - 1) / ns + 15) / 16 * 16;
    if (ns > 1 && kc < 512) break;
    const double rounds = (double)((tiles * ns + conc - 1) / conc);
    const double t = rounds * (double)kc * us_per_k +
                     (ns > 1 ? (double)ns * (double)MN * 16.0 / 4e6 : 0.0);
    if (t < tbest * 0.98) { tbest = t; best = ns; }
  }
  return best;
}

// Autotuner of the K split.  The first time a large single product of a given
// shape (precision, transposes, M, N, K) runs, the split chosen by the model
// above and its neighbours (1, s/2, 2s) are each timed once with HIP events
// into a scratch output, and the fastest is kept for the rest of the process;
// the real product then runs once with that split.  NACME_AUTOTUNE=0 keeps
// the model's choice.
static std::mutex g_tune_mu;
static std::map<std::string, int64_t> g_tune;
static bool autotune_on() {
  const char* e = std::getenv("NACME_AUTOTUNE");
  return !(e && e[0] == '0');
}
static std::string tune_key(char prec, bool ta, bool tb, int64_t M, int64_t N, int64_t K) {
  return std::string(1, prec) + (ta ? "T" : "N") + (tb ? "T" : "N") + ":" + std::to_string(M) + "x" +
         std::to_string(N) + "x" + std::to_string(K);
}
// times launch(c) for each candidate configuration c (outputs go to scratch)
// and returns the fastest; the first candidate is the model's choice
static int64_t tune_config(hipStream_t s, const std::string& key, std::vector<int64_t> cand,
                           const std::function<void(int64_t)>& launch) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  const int64_t model = cand.front();
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  int64_t best = model;
  float tbest = 1e30f;
  for (int64_t c : cand) {
    hip_check(hipEventRecord(e0, s), "event");
    launch(c);
    hip_check(hipEventRecord(e1, s), "event");
    hip_check(hipEventSynchronize(e1), "event");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
    if (ms < tbest) { tbest = ms; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (std::getenv("NACME_VERBOSE"))
    std::fprintf(stderr, "[autotune] %s config %lld (model %lld) %.3f ms\n", key.c_str(),
                 (long long)best, (long long)model, tbest);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  return best;
}

// K split only: the model's split and its neighbours (no split at all only
// near a small model split: for the skinny long-K products, model splits in
// the hundreds, one chunk takes seconds)
static int64_t tune_split(hipStream_t s, const std::string& key, int64_t model, int64_t ns_max,
                          const std::function<void(int64_t)>& launch) {
  std::vector<int64_t> cand{model, std::max<int64_t>(1, model / 2), std::min<int64_t>(ns_max, model * 2)};
  if (model <= 16) cand.push_back(1);
  return tune_config(s, key, cand, launch);
}
static constexpr double kTuneMinFlops = 2e10;

// Can `v` be read as a (batched) row-major matrix rows x cols with a leading
// dimension?  cols must be compact with unit innermost stride; rows must be
// nested uniformly with the last row stride = ld; batch labels nested above.
static bool as_matrix(const DView& v, const std::string& batch, const std::string& rows,
                      const std::string& cols, int64_t& ld, int64_t& bstride) {
  int64_t s = 1;
  for (int k = (int)cols.size() - 1; k >= 0; --k) {
    const int d = find_lab(v, cols[k]);
    if (d < 0) return false;
    if (v.dims[d] != 1 && v.str[d] != s) return false;
    s *= v.dims[d];
  }
  const int64_t ncols = s;
  if (rows.empty()) {
    ld = std::max<int64_t>(ncols, 1);
    s = ld;
  } else {
    const int dl = find_lab(v, rows.back());
    if (dl < 0) return false;
    ld = v.dims[dl] == 1 ? std::max<int64_t>(ncols, 1) : v.str[dl];
    if (ld < ncols) return false;
    s = ld;
    for (int k = (int)rows.size() - 1; k >= 0; --k) {
      const int d = find_lab(v, rows[k]);
      if (d < 0) return false;
      if (v.dims[d] != 1 && v.str[d] != s) return false;
      s *= v.dims[d];
    }
  }
  // batch labels: nested uniformly (any outer stride)
  if (batch.empty()) {
    bstride = s;
    return true;
  }
  const int db = find_lab(v, batch.back());
  if (db < 0) return false;
  bstride = v.str[db];
  if (v.dims[db] != 1 && bstride < s) return false;
  int64_t t = bstride;
  for (int k = (int)batch.size() - 1; k >= 0; --k) {
    const int d = find_lab(v, batch[k]);
    if (d < 0) return false;
    if (v.dims[d] != 1 && v.str[d] != t) return false;
    t *= v.dims[d];
  }
  return true;
}

static int64_t prod_of(const DView& v, const std::string& s) {
  int64_t p = 1;
  for (char c : s) p *= v.dims[find_lab(v, c)];
  return p;
}

static std::string labels_of(const DView& v) { return std::string(v.lab, v.lab + v.nd); }

__global__ void scalar_axpy_kernel(double* y, const double* x, double a) { *y += a * (*x); }

// The same values with the labels of the two index halves exchanged (valid
// for pair-symmetric tensors).
static DView swap_halves(const DView& v) {
  DView w = v;
  const int h = v.nd / 2;
  for (int k = 0; k < v.nd; ++k) w.lab[k] = v.lab[(k + h) % v.nd];
  return w;
}
static bool halves_match(const DView& v) {
  if (!v.pair_sym || v.nd % 2 != 0 || v.nd == 0) return false;
  for (int k = 0; k < v.nd; ++k)
    if (v.dims[k] != v.dims[(k + v.nd / 2) % v.nd]) return false;
  return true;
}

// fp32 copy of `src` laid out row-major in label order `order`; constant
// sources are converted once and kept (up to 8 GB), others go to the arena.
static ViewSpec pack_spec(const DView& src, const std::string& order, int64_t& count) {
  ViewSpec vs;
  vs.nd = (int)order.size();
  int64_t st = 1;
  for (int k = vs.nd - 1; k >= 0; --k) {
    const int j = find_lab(src, order[k]);
    vs.dims[k] = src.dims[j];
    vs.ostr[k] = st;
    vs.istr[k] = src.str[j];
    st *= src.dims[j];
  }
  count = st;
  return vs;
}

const float* Engine::packed_f32(const DView& src, const std::string& order, bool cache) {
  int64_t cnt = 0;
  const ViewSpec vs = pack_spec(src, order, cnt);
  if (src.constant && cache) {
    std::string key = std::to_string((uintptr_t)src.p);
    for (int k = 0; k < vs.nd; ++k)
      key += ":" + std::to_string(vs.dims[k]) + "/" + std::to_string(vs.istr[k]);
    auto it = f32_cache_.find(key);
    if (it != f32_cache_.end()) return it->second;
    const size_t bytes = (size_t)cnt * sizeof(float);
    if (f32_cache_bytes_ + bytes <= ((size_t)8 << 30)) {
      float* buf = nullptr;
      if (hipMalloc((void**)&buf, bytes) == hipSuccess) {
        kcheck(view_gather_f32(s_, buf, src.p, vs), "pack fp32");
        f32_cache_[key] = buf;
        f32_cache_bytes_ += bytes;
        return buf;
      }
      (void)hipGetLastError();
    }
  }
  if (src.frozen && cache) {
    std::string key = "f" + std::to_string((uintptr_t)src.p);
    for (int k = 0; k < vs.nd; ++k)
      key += ":" + std::to_string(vs.dims[k]) + "/" + std::to_string(vs.istr[k]);
    if (void* hit = frozen_lookup(key)) return (const float*)hit;
    if (float* buf = (float*)frozen_store(key, (size_t)cnt * sizeof(float))) {
      kcheck(view_gather_f32(s_, buf, src.p, vs), "pack fp32");
      return buf;
    }
  }
  float* buf = (float*)arena_.alloc((cnt + 1) / 2);
  kcheck(view_gather_f32(s_, buf, src.p, vs), "pack fp32");
  return buf;
}

void Engine::packed_bf16(const DView& src, const std::string& order, int64_t rows, int64_t K,
                         int64_t Kp, const uint16_t** pairs) {
  std::string key;
  if (src.constant || src.frozen) {
    int64_t cnt = 0;
    const ViewSpec vs = pack_spec(src, order, cnt);
    key = std::to_string((uintptr_t)src.p) + ":" + std::to_string(Kp);
    for (int k = 0; k < vs.nd; ++k)
      key += ":" + std::to_string(vs.dims[k]) + "/" + std::to_string(vs.istr[k]);
  }
  const size_t n = (size_t)(rows * Kp);
  if (src.constant) {
    auto it = bf16_cache_.find(key);
    if (it != bf16_cache_.end()) {
      *pairs = it->second;
      return;
    }
  } else if (src.frozen) {
    if (void* hit = frozen_lookup("h" + key)) {
      *pairs = (const uint16_t*)hit;
      return;
    }
  }
  uint16_t* buf = nullptr;
  bool cached = false;
  if (src.constant && bf16_cache_bytes_ + 2 * n * sizeof(uint16_t) <= ((size_t)8 << 30)) {
    if (hipMalloc((void**)&buf, 2 * n * sizeof(uint16_t)) == hipSuccess) {
      cached = true;
    } else {
      (void)hipGetLastError();
      buf = nullptr;
    }
  } else if (src.frozen) {
    buf = (uint16_t*)frozen_store("h" + key, 2 * n * sizeof(uint16_t));
  }
  if (!buf) buf = (uint16_t*)arena_.alloc((int64_t)((2 * n * sizeof(uint16_t) + 7) / 8));
  // one pass from the fp64 view: output strides of the trailing K labels as
  // packed, those of the leading (row) labels scaled from K to Kp
  int64_t cnt = 0;
  ViewSpec vs = pack_spec(src, order, cnt);
  int nk = 0;
  for (int64_t p = 1; nk < vs.nd && p < K; ++nk) p *= vs.dims[vs.nd - 1 - nk];
  if (nk == 0 && K == 1) nk = 1;
  for (int d = 0; d < vs.nd - nk; ++d) vs.ostr[d] = vs.ostr[d] / K * Kp;
  kcheck(view_gather_bf16x2(s_, buf, src.p, vs, rows, (int)K, (int)Kp), "pack bf16 pairs");
  if (cached) {
    bf16_cache_[key] = buf;
    bf16_cache_bytes_ += 2 * n * sizeof(uint16_t);
  }
  *pairs = buf;
}

void Engine::contract(double alpha, const DView& A_in, const DView& B_in, const DView& C,
                      bool overwrite) {
  TermTrace trace(s_, lowp_ ? (bf16_ ? "mul16x3" : "mul32") : "mul", A_in, &B_in, C);
  // A pair-symmetric operand whose contracted labels sit in its leading half
  // is relabelled so that they sit in the trailing half (B: leading), which
  // turns a transposed GEMM operand into a plain one.
  DView A = A_in, B = B_in;
  auto in_half = [](const DView& v, const DView& other, bool lead) {
    const int h = v.nd / 2;
    for (int k = lead ? 0 : h; k < (lead ? h : v.nd); ++k)
      if (find_lab(other, v.lab[k]) < 0) return false;
    return true;
  };
  if (halves_match(B) && in_half(B, A, false) && !in_half(B, A, true)) B = swap_halves(B);
  if (halves_match(A) && in_half(A, B, true) && !in_half(A, B, false)) A = swap_halves(A);
  std::string sb, sm, sn, sk;
  for (int k = 0; k < A.nd; ++k) {
    const char c = A.lab[k];
    const bool inB = find_lab(B, c) >= 0, inC = find_lab(C, c) >= 0;
    if (inB && inC) sb += c;
    else if (inC) sm += c;
    else if (inB) sk += c;
    else throw Error(-1, std::string("label '") + c + "' only in first operand");
  }
  for (int k = 0; k < B.nd; ++k) {
    const char c = B.lab[k];
    const bool inA = find_lab(A, c) >= 0, inC = find_lab(C, c) >= 0;
    if (!inA && inC) sn += c;
    else if (!inA) throw Error(-1, std::string("label '") + c + "' only in second operand");
  }
  for (int k = 0; k < C.nd; ++k)
    if (find_lab(A, C.lab[k]) < 0 && find_lab(B, C.lab[k]) < 0)
      throw Error(-1, "output label in neither operand");
  for (char c : sk)
    if (A.dims[find_lab(A, c)] != B.dims[find_lab(B, c)]) throw Error(-1, "contracted dim mismatch");
  for (char c : sb)
    if (A.dims[find_lab(A, c)] != B.dims[find_lab(B, c)]) throw Error(-1, "batch dim mismatch");
  const int64_t nb0 = prod_of(A, sb), M0 = prod_of(A, sm), N0 = prod_of(B, sn), K = prod_of(A, sk);
  if (nb0 == 0 || M0 == 0 || N0 == 0) return;
  flops_ += (uint64_t)(2.0 * (double)nb0 * (double)M0 * (double)N0 * (double)K);
  if (K == 0) return;
  Arena::Mark mk = arena_.mark();

  // Full contraction to a scalar: deterministic dot product.
  if (C.nd == 0 && sb.empty()) {
    const std::string ord = sk;
    const double* pa = contiguous_in(A, ord) ? A.p : packed_view(arena_, A, ord, s_).p;
    const double* pb = contiguous_in(B, ord) ? B.p : packed_view(arena_, B, ord, s_).p;
    double* tmp = scalar_slot(63);
    kcheck(dot(s_, pa, pb, K, 1, 1, 0, red_, tmp), "dot");
    if (overwrite) kcheck(fill(s_, C.p, 0.0, 1), "fill");
    hipLaunchKernelGGL(scalar_axpy_kernel, dim3(1), dim3(1), 0, s_, C.p, tmp, alpha);
    kcheck(hipGetLastError() == hipSuccess ? 0 : -3, "scalar axpy");
    arena_.rewind(mk);
    return;
  }

  // A product of a large operand X with a small one F over a short contracted
  // range (K < 64: the occupied-index sums) is bound by memory, so it runs in
  // fp64 in both precisions, as a batched GEMM that reads X and updates C in
  // place with F packed transposed ([n][k], a few KB):
  //   C_b[n][r] = sum_k F[k][n] X_b[k][r],
  // b = leading labels of X that also lead C, r = the other labels of X that
  // C holds (trailing both), n = F's labels in C.  Layouts that do not allow
  // it fall through to the general paths.
  if (sb.empty() && K < 64) {
    const int64_t na = prod_of(A, labels_of(A)), nbv = prod_of(B, labels_of(B));
    const bool smallB = nbv <= ((int64_t)1 << 16) && na >= ((int64_t)1 << 20);
    const bool smallA = na <= ((int64_t)1 << 16) && nbv >= ((int64_t)1 << 20);
    if (smallA || smallB) {
      const DView& X = smallB ? A : B;
      const DView& F = smallB ? B : A;
      std::string kx, rx, nc;
      for (int d = 0; d < X.nd; ++d) (find_lab(C, X.lab[d]) >= 0 ? rx : kx) += X.lab[d];
      for (int d = 0; d < C.nd; ++d)
        if (find_lab(X, C.lab[d]) < 0) nc += C.lab[d];
      for (int L = std::min(X.nd, C.nd); L >= 0; --L) {
        const std::string pre(X.lab, X.lab + L);
        if (std::string(C.lab, C.lab + L) != pre) continue;
        std::string rest;
        for (char ch : rx)
          if (pre.find(ch) == std::string::npos) rest += ch;
        int64_t ldx, bsx, ldcs, bsc;
        if (rest.empty() || prod_of(X, rest) < 16 || !as_matrix(X, pre, kx, rest, ldx, bsx) ||
            !as_matrix(C, pre, nc, rest, ldcs, bsc))
          continue;
        const int64_t Mn = prod_of(F, nc), Nr = prod_of(X, rest), nbx = prod_of(X, pre);
        if (Mn > INT32_MAX || Nr > INT32_MAX || nbx > INT32_MAX) break;
        const DView Fp = packed_view(arena_, F, nc + kx, s_);
        kcheck(gemm_f64(s_, false, false, (int)Mn, (int)Nr, (int)K, (int)nbx, alpha, Fp.p, K, 0, X.p,
                        ldx, bsx, overwrite ? 0.0 : 1.0, C.p, ldcs, bsc),
               "gemm (small operand)");
        arena_.rewind(mk);
        return;
      }
      // no GEMM-shaped layout without copies: the short-K kernels read the
      // views as they are
      if (smallk_contract(s_, alpha, X, F, C, overwrite)) {
        arena_.rewind(mk);
        return;
      }
    }
  }

  // Mixed-precision path for large contractions: pack both operands to fp32
  // in [batch][rows][k] / [batch][k][cols] order and multiply on the FP32
  // matrix cores (fp32 accumulation, fp64 result); products with few output
  // tiles and a long K are split over K like the fp64 path.
  // (batched products only when each product fills most of a 128 x 128 tile)
  if (lowp_ && K >= 4 && M0 * N0 >= 16 && (sb.empty() || (M0 >= 96 && N0 >= 96)) &&
      2.0 * (double)nb0 * (double)M0 * (double)N0 * (double)K >= lowp_min_flops_) {
    if (M0 > INT32_MAX || N0 > INT32_MAX || K > INT32_MAX || nb0 > INT32_MAX)
      throw Error(-1, "GEMM dimension overflow");
    // bf16 pairs: A as [batch][rows][2 Kp], B transposed as [batch][cols][2 Kp]
    // (hi and lo interleaved in 16-byte chunks)
    const bool use_bf16 = bf16_ && K >= 32;
    const int64_t Kp = (K + 31) / 32 * 32;
    const float* a32 = nullptr;
    const float* b32 = nullptr;
    const uint16_t *ap = nullptr, *bp = nullptr;
    if (use_bf16) {
      packed_bf16(A, sb + sm + sk, nb0 * M0, K, Kp, &ap);
      packed_bf16(B, sb + sn + sk, nb0 * N0, K, Kp, &bp);
    } else {
      a32 = packed_f32(A, sb + sm + sk);
      b32 = packed_f32(B, sb + sk + sn);
    }
    int64_t ldc, sC;
    const bool direct = as_matrix(C, sb, sm, sn, ldc, sC);
    double* pc;
    DView cbuf;
    if (direct) {
      pc = C.p;
    } else {
      const std::string ord = sb + sm + sn;
      cbuf.nd = (int)ord.size();
      int64_t st = 1;
      for (int k = cbuf.nd - 1; k >= 0; --k) {
        const char ch = ord[k];
        const int ja = find_lab(A, ch);
        cbuf.lab[k] = ch;
        cbuf.dims[k] = ja >= 0 ? A.dims[ja] : B.dims[find_lab(B, ch)];
        cbuf.str[k] = st;
        st *= cbuf.dims[k];
      }
      cbuf.p = arena_.alloc(st);
      pc = cbuf.p;
      ldc = N0;
      sC = M0 * N0;
    }
    const double a_ = direct ? alpha : 1.0, b_ = (direct && !overwrite) ? 1.0 : 0.0;
    const int64_t tiles = ((M0 + 127) / 128) * ((N0 + 127) / 128) * nb0;
    int64_t ns = 1;
    if (nb0 == 1 && tiles < 256 && K >= 2048) {
      ns = std::min<int64_t>(std::max<int64_t>(1, 512 / tiles), K / 512);
      ns = std::max<int64_t>(1, std::min<int64_t>(ns, 256));
    } else if (nb0 == 1) {
      ns = big_split(tiles, K, M0 * N0, use_bf16 ? kBF16UsPerK : kF32UsPerK);
    }
    // bf16 pairs: a configuration is tile shape * kCfgTile + K split
    constexpr int64_t kCfgTile = 1024;
    int bf16_tile = use_bf16 ? bf16x3_auto_tile((int)M0, (int)N0, (int)nb0) : 0;
    auto launch = [&](int64_t cfg, double* out, int64_t ldo, int64_t so, double aa, double bb) {
      if (use_bf16) {
        const int tile = (int)(cfg / kCfgTile);
        const int64_t nsplit = cfg % kCfgTile;
        if (nsplit > 1) {
          const int64_t kc = ((Kp + nsplit - 1) / nsplit + 31) / 32 * 32;
          const int64_t nsr = (Kp + kc - 1) / kc;
          const int64_t klast = Kp - (nsr - 1) * kc;
          Arena::Mark pm = arena_.mark();
          double* part = arena_.alloc(nsr * M0 * N0);
          kcheck(gemm_bf16x3(s_, (int)M0, (int)N0, (int)kc, (int)nsr, 1.0, ap, 2 * Kp, 2 * kc, bp, 2 * Kp,
                             2 * kc, 0.0, part, N0, M0 * N0, (int)klast, tile),
                 "gemm bf16x3 (split K)");
          const int64_t tot = M0 * N0;
          const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
          hipLaunchKernelGGL(splitk_fold_kernel, dim3(g), dim3(256), 0, s_, out, ldo, part, (int)M0,
                             (int)N0, (int)nsr, aa, bb);
          kcheck(hipGetLastError() == hipSuccess ? 0 : -3, "splitk fold");
          arena_.rewind(pm);
        } else {
          kcheck(gemm_bf16x3(s_, (int)M0, (int)N0, (int)Kp, (int)nb0, aa, ap, 2 * Kp, 2 * M0 * Kp, bp,
                             2 * Kp, 2 * N0 * Kp, bb, out, ldo, so, 0, tile),
                 "gemm bf16x3");
        }
        return;
      }
      const int64_t nsplit = cfg;
      if (nsplit > 1) {
        const int64_t kc = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
        const int64_t nsr = (K + kc - 1) / kc;
        const int64_t klast = K - (nsr - 1) * kc;
        Arena::Mark pm = arena_.mark();
        double* part = arena_.alloc(nsr * M0 * N0);
        kcheck(gemm_f32acc(s_, false, false, (int)M0, (int)N0, (int)kc, (int)nsr, 1.0, a32, K, kc,
                           b32, N0, kc * N0, 0.0, part, N0, M0 * N0, (int)klast),
               "gemm fp32 (split K)");
        const int64_t tot = M0 * N0;
        const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
        hipLaunchKernelGGL(splitk_fold_kernel, dim3(g), dim3(256), 0, s_, out, ldo, part, (int)M0,
                           (int)N0, (int)nsr, aa, bb);
        kcheck(hipGetLastError() == hipSuccess ? 0 : -3, "splitk fold");
        arena_.rewind(pm);
      } else {
        kcheck(gemm_f32acc(s_, false, false, (int)M0, (int)N0, (int)K, (int)nb0, aa, a32, K, M0 * K,
                           b32, N0, K * N0, bb, out, ldo, so),
               "gemm fp32");
      }
    };
    int64_t cfg = use_bf16 ? bf16_tile * kCfgTile + ns : ns;
    if (nb0 == 1 && autotune_on() && 2.0 * (double)M0 * (double)N0 * (double)K >= kTuneMinFlops) {
      double* scratch = arena_.alloc(M0 * N0);
      auto run = [&](int64_t c) { launch(c, scratch, N0, M0 * N0, 1.0, 0.0); };
      if (use_bf16) {
        // every tile shape with its own modelled split (one workgroup per CU
        // for the large tiles), and the neighbours of the chosen split
        std::vector<int64_t> cand{cfg, bf16_tile * kCfgTile + std::max<int64_t>(1, ns / 2),
                                  bf16_tile * kCfgTile + std::min<int64_t>(256, ns * 2)};
        for (int t = 0; t < kBf16Tiles; ++t) {
          int tbm, tbn;
          bf16x3_tile_dims(t, tbm, tbn);
          const int64_t bm = tbm, bn = tbn;
          const int64_t tt = ((M0 + bm - 1) / bm) * ((N0 + bn - 1) / bn);
          // a large-tile workgroup holds a whole CU and, by the model, moves
          // 1.8x the outputs per cycle of two 128 x 128 workgroups
          const double upk = t == 0 ? kBF16UsPerK
                                    : kBF16UsPerK * (double)(bm * bn) / (2.0 * 16384.0) / 1.8;
          const int64_t st = big_split(tt, K, M0 * N0, upk, t == 0 ? 512 : 256);
          cand.push_back(t * kCfgTile + st);
        }
        cfg = tune_config(s_, tune_key('h', false, false, M0, N0, K), cand, run);
      } else {
        cfg = tune_split(s_, tune_key('s', false, false, M0, N0, K), ns, 256, run);
      }
    }
    launch(cfg, pc, ldc, sC, a_, b_);
    if (!direct) gather_into(s_, alpha, cbuf, C, overwrite ? 0.0 : 1.0);
    lowp_flops_ += (uint64_t)(2.0 * (double)nb0 * (double)M0 * (double)N0 * (double)K);
    arena_.rewind(mk);
    return;
  }

  // Promote outer labels shared by C and B (N labels) or by C and A (M labels)
  // to a batch dimension with a broadcast (stride 0) other operand.
  std::string pb_lab, pa_lab;   // promoted labels
  if (sb.empty()) {
    const std::string cl = labels_of(C), bl = labels_of(B), al = labels_of(A);
    std::string cand;
    for (size_t k = 0; k < cl.size() && k < bl.size(); ++k) {
      if (cl[k] != bl[k] || sn.find(cl[k]) == std::string::npos) break;
      cand += cl[k];
    }
    std::string candA;
    for (size_t k = 0; k < cl.size() && k < al.size(); ++k) {
      if (cl[k] != al[k] || sm.find(cl[k]) == std::string::npos) break;
      candA += cl[k];
    }
    auto strip = [](std::string s, const std::string& rm) {
      std::string r;
      for (char c : s)
        if (rm.find(c) == std::string::npos) r += c;
      return r;
    };
    int64_t ld, bs;
    // only promote when the unpromoted layout would need a copy
    // ba / bb: batch labels as seen by A / B (empty for the broadcast operand)
    auto direct_ok = [&](const std::string& ba, const std::string& bb, const std::string& bc,
                         const std::string& m, const std::string& n) {
      return (as_matrix(A, ba, m, sk, ld, bs) || as_matrix(A, ba, sk, m, ld, bs)) &&
             (as_matrix(B, bb, sk, n, ld, bs) || as_matrix(B, bb, n, sk, ld, bs)) &&
             as_matrix(C, bc, m, n, ld, bs);
    };
    // copies the unpromoted layout would need (doubles)
    int64_t copy_cost = 0;
    if (!(as_matrix(A, "", sm, sk, ld, bs) || as_matrix(A, "", sk, sm, ld, bs))) copy_cost += M0 * K;
    if (!(as_matrix(B, "", sk, sn, ld, bs) || as_matrix(B, "", sn, sk, ld, bs))) copy_cost += K * N0;
    if (!as_matrix(C, "", sm, sn, ld, bs)) copy_cost += M0 * N0;
    // promote only when it saves a large copy and leaves a GEMM-shaped batch
    if (copy_cost > (int64_t)1 << 22) {
      for (size_t len = cand.size(); len > 0 && pb_lab.empty(); --len) {
        const std::string pre = cand.substr(0, len);
        if (N0 / prod_of(B, pre) >= 16 && direct_ok("", pre, pre, sm, strip(sn, pre))) pb_lab = pre;
      }
      if (pb_lab.empty())
        for (size_t len = candA.size(); len > 0 && pa_lab.empty(); --len) {
          const std::string pre = candA.substr(0, len);
          if (M0 / prod_of(A, pre) >= 16 && direct_ok(pre, "", pre, strip(sm, pre), sn)) pa_lab = pre;
        }
    }
    if (!pb_lab.empty()) {
      sb = pb_lab;
      sn = strip(sn, pb_lab);
    } else if (!pa_lab.empty()) {
      sb = pa_lab;
      sm = strip(sm, pa_lab);
    }
  }
  // contracted labels in the memory order of the larger operand when that
  // lets it be read in place (the smaller one is packed instead)
  if (sk.size() > 1) {
    const bool bigB = prod_of(B, labels_of(B)) > prod_of(A, labels_of(A));
    const DView& Big = bigB ? B : A;
    std::string sko;
    for (int d = 0; d < Big.nd; ++d)
      if (sk.find(Big.lab[d]) != std::string::npos) sko += Big.lab[d];
    if (sko != sk) {
      int64_t l_, s_b;
      const std::string bbig = bigB ? (!pa_lab.empty() ? "" : sb) : (!pb_lab.empty() ? "" : sb);
      const std::string& free_ = bigB ? sn : sm;
      const bool in_place_now = as_matrix(Big, bbig, sk, free_, l_, s_b) || as_matrix(Big, bbig, free_, sk, l_, s_b);
      const bool in_place_new = as_matrix(Big, bbig, sko, free_, l_, s_b) || as_matrix(Big, bbig, free_, sko, l_, s_b);
      if (!in_place_now && in_place_new) sk = sko;
    }
  }
  const bool bcastA = !pb_lab.empty(), bcastB = !pa_lab.empty();
  const int64_t nb = bcastA ? prod_of(B, sb) : prod_of(A, sb);
  const int64_t M = prod_of(A, sm), N = prod_of(B, sn);

  bool ta = false, tb = false;
  const double* pa;
  const double* pb;
  int64_t lda, ldb, sA, sB;
  const std::string sbA = bcastA ? "" : sb, sbB = bcastB ? "" : sb;
  if (as_matrix(A, sbA, sm, sk, lda, sA)) { pa = A.p; }
  else if (as_matrix(A, sbA, sk, sm, lda, sA)) { pa = A.p; ta = true; }
  else { DView p = packed_view(arena_, A, sbA + sm + sk, s_); pa = p.p; lda = K; sA = M * K; }
  if (as_matrix(B, sbB, sk, sn, ldb, sB)) { pb = B.p; }
  else if (as_matrix(B, sbB, sn, sk, ldb, sB)) { pb = B.p; tb = true; }
  else { DView p = packed_view(arena_, B, sbB + sk + sn, s_); pb = p.p; ldb = N; sB = K * N; }
  if (bcastA) sA = 0;
  if (bcastB) sB = 0;

  int64_t ldc, sC;
  const bool direct = as_matrix(C, sb, sm, sn, ldc, sC);
  double* pc;
  DView cbuf;
  if (direct) {
    pc = C.p;
  } else {
    const std::string ord = sb + sm + sn;
    cbuf.nd = (int)ord.size();
    int64_t st = 1;
    for (int k = cbuf.nd - 1; k >= 0; --k) {
      const char c = ord[k];
      const int ja = find_lab(A, c);
      cbuf.lab[k] = c;
      cbuf.dims[k] = ja >= 0 ? A.dims[ja] : B.dims[find_lab(B, c)];
      cbuf.str[k] = st;
      st *= cbuf.dims[k];
    }
    cbuf.p = arena_.alloc(st);
    pc = cbuf.p;
    ldc = N;
    sC = M * N;
  }
  const double a_ = direct ? alpha : 1.0, b_ = (direct && !overwrite) ? 1.0 : 0.0;
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) throw Error(-1, "GEMM dimension overflow");

  const bool big = M >= 128 && N >= 128;   // gemm_f64 then runs 128 x 128 tiles
  const int64_t tiles = big ? ((M + 127) / 128) * ((N + 127) / 128) * nb
                            : ((M + 63) / 64) * ((N + 63) / 64) * nb;
  // K split of one product (pointers of batch entry b): split-K GEMM in one
  // launch (K chunks on grid.z, the last possibly shorter), partials folded
  // in a fixed order
  int64_t ns = 1;
  if (big) {
    if (nb == 1) ns = big_split(tiles, K, M * N, kF64UsPerK);
  } else if (tiles < 512 && K >= 4096) {
    // skinny products with a long K (gradients of the integral transforms):
    // enough K chunks for ~4096 workgroups of at least 512 K each, partials
    // capped at 2^26 doubles
    ns = std::min<int64_t>(std::max<int64_t>(1, 4096 / tiles), K / 512);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, ((int64_t)1 << 26) / (M * N)));
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, 2048));
  }
  // a few batch entries that leave the device idle are run one by one,
  // each split over K
  if (nb > 64) ns = 1;
  // the product with K split in `nsplit` chunks into out (ld ldo, batch stride so)
  auto launch = [&](int64_t nsplit, double* out, int64_t ldo, int64_t so, double aa, double bb) {
    if (nsplit > 1) {
      const int64_t kc = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
      const int64_t nsr = (K + kc - 1) / kc;
      Arena::Mark pm = arena_.mark();
      double* part = arena_.alloc(nsr * M * N);
      const int64_t klast = K - (nsr - 1) * kc;
      for (int64_t b = 0; b < nb; ++b) {
        kcheck(gemm_f64(s_, ta, tb, (int)M, (int)N, (int)kc, (int)nsr, 1.0, pa + b * sA, lda,
                        ta ? kc * lda : kc, pb + b * sB, ldb, tb ? kc : kc * ldb, 0.0, part, N,
                        M * N, (int)klast),
               "gemm(splitk)");
        const int64_t tot = M * N;
        const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
        hipLaunchKernelGGL(splitk_fold_kernel, dim3(g), dim3(256), 0, s_, out + b * so, ldo, part,
                           (int)M, (int)N, (int)nsr, aa, bb);
        kcheck(hipGetLastError() == hipSuccess ? 0 : -3, "splitk fold");
      }
      arena_.rewind(pm);
    } else {
      kcheck(gemm_f64(s_, ta, tb, (int)M, (int)N, (int)K, (int)nb, aa, pa, lda, sA, pb, ldb, sB, bb,
                      out, ldo, so),
             "gemm");
    }
  };
  if (nb == 1 && autotune_on() && 2.0 * (double)M * (double)N * (double)K >= kTuneMinFlops) {
    double* scratch = arena_.alloc(M * N);
    ns = tune_split(s_, tune_key('d', ta, tb, M, N, K), ns, big ? 256 : 2048,
                    [&](int64_t c) { launch(c, scratch, N, M * N, 1.0, 0.0); });
  }
  launch(ns, pc, ldc, sC, a_, b_);
  if (!direct) gather_into(s_, alpha, cbuf, C, overwrite ? 0.0 : 1.0);
  arena_.rewind(mk);
}

// ------------------------------------------------------------------- Graph
Graph::~Graph() {}

int Graph::leaf(const Tensor& t) {
  Node n;
  n.val = t;
  n.leaf = true;
  nodes_.push_back(n);
  return (int)nodes_.size() - 1;
}

DView Graph::view_of(const Op& o, const Tensor& t) const {
  if ((int)o.lab.size() != t.nd) throw Error(-1, "operand label count != tensor rank");
  if (!o.box.empty() && (int)o.box.size() != t.nd) throw Error(-1, "operand box rank mismatch");
  int64_t st[kMaxViewDims];
  strides_of(t, st);
  DView v;
  int64_t base = 0;
  for (int k = 0; k < t.nd; ++k) {
    const int64_t lo = o.box.empty() ? 0 : o.box[k].lo;
    const int64_t len = o.box.empty() ? t.d[k] : o.box[k].len;
    if (lo < 0 || lo + len > t.d[k]) throw Error(-1, "operand box out of range");
    base += lo * st[k];
    const int j = find_lab(v, o.lab[k]);
    if (j >= 0) {
      if (v.dims[j] != len) throw Error(-1, "repeated label with different extents");
      v.str[j] += st[k];
    } else {
      v.lab[v.nd] = o.lab[k];
      v.dims[v.nd] = len;
      v.str[v.nd] = st[k];
      v.nd++;
    }
  }
  v.p = t.p + base;
  v.pair_sym = t.pair_sym && o.box.empty() && v.nd == t.nd;
  v.constant = t.constant;
  v.frozen = t.frozen;
  return v;
}

DView Graph::out_view(const Term& tm, const Tensor& t) const {
  Op o;
  o.lab = tm.olab;
  o.box = tm.obox;
  DView v = view_of(o, t);
  if (v.nd != t.nd) throw Error(-1, "output labels must be distinct");
  return v;
}

int Graph::node(const std::vector<int64_t>& shape, const std::vector<Term>& terms) {
  Node n;
  // The first term may overwrite the (uninitialised) output when it covers
  // the whole node and is not a broadcast.
  bool first_overwrites = false;
  if (!terms.empty() && terms[0].obox.empty()) {
    const Term& t0 = terms[0];
    if (t0.bilinear) {
      first_overwrites = true;
    } else {
      first_overwrites = true;
      for (char ch : t0.olab)
        if (t0.a.lab.find(ch) == std::string::npos) first_overwrites = false;
    }
  }
  n.val = make_tensor(e_.arena(), shape, !first_overwrites, e_.stream());
  n.terms = terms;
  bool first = true;
  for (const Term& tm : terms) {
    DView C = out_view(tm, n.val);
    DView A = view_of(tm.a, nodes_.at(tm.a.node).val);
    const bool ow = first && first_overwrites;
    first = false;
    if (tm.bilinear) {
      DView B = view_of(tm.b, nodes_.at(tm.b.node).val);
      e_.contract(tm.alpha, A, B, C, ow);
    } else {
      e_.linear(tm.alpha, A, C, ow);
    }
  }
  nodes_.push_back(n);
  return (int)nodes_.size() - 1;
}

// Batched derivatives: tangents / adjoints of `nb` directions at once carry
// a leading batch index with label kBatchLabel on the derivative operand and
// on the output of every term (the primal operand is shared by the batch).
static constexpr char kBatchLabel = 'Z';
static Op batched_op(Op o, int64_t nb) {
  if (nb <= 0) return o;
  o.lab.insert(o.lab.begin(), kBatchLabel);
  if (!o.box.empty()) o.box.insert(o.box.begin(), Range{0, nb});
  return o;
}
static Term batched_out(Term t, int64_t nb) {
  if (nb <= 0) return t;
  t.olab.insert(t.olab.begin(), kBatchLabel);
  if (!t.obox.empty()) t.obox.insert(t.obox.begin(), Range{0, nb});
  return t;
}
static std::vector<int64_t> batched_shape(std::vector<int64_t> s, int64_t nb) {
  if (nb > 0) s.insert(s.begin(), nb);
  return s;
}

std::map<int, int> Graph::jvp(const std::map<int, int>& seeds, int first, int64_t batch) {
  std::map<int, int> tan = seeds;
  const int end = (int)nodes_.size();
  for (int k = first; k < end; ++k) {
    if (tan.count(k)) continue;
    const Node nk = nodes_[k];   // copy: nodes_ grows below
    if (nk.leaf) continue;
    std::vector<Term> tt;
    for (const Term& tm : nk.terms) {
      auto ia = tan.find(tm.a.node);
      if (tm.bilinear) {
        auto ib = tan.find(tm.b.node);
        if (ia != tan.end()) {
          Term x = batched_out(tm, batch);
          x.a = batched_op(tm.a, batch);
          x.a.node = ia->second;
          tt.push_back(x);
        }
        if (ib != tan.end()) {
          Term x = batched_out(tm, batch);
          x.b = batched_op(tm.b, batch);
          x.b.node = ib->second;
          tt.push_back(x);
        }
      } else if (ia != tan.end()) {
        Term x = batched_out(tm, batch);
        x.a = batched_op(tm.a, batch);
        x.a.node = ia->second;
        tt.push_back(x);
      }
    }
    if (!tt.empty()) tan[k] = node(batched_shape(nk.val.shape(), batch), tt);
  }
  return tan;
}

std::map<int, Tensor> Graph::vjp(const std::map<int, const double*>& seeds,
                                 const std::vector<int>& wrt, int64_t batch) {
  const int n = (int)nodes_.size();
  std::vector<char> needs(n, 0);
  for (int w : wrt) needs.at(w) = 1;
  for (int k = 0; k < n; ++k) {
    if (needs[k]) continue;
    for (const Term& tm : nodes_[k].terms) {
      if (needs[tm.a.node] || (tm.bilinear && needs[tm.b.node])) {
        needs[k] = 1;
        break;
      }
    }
  }
  std::vector<Tensor> adj(n);
  auto get_adj = [&](int k) -> Tensor& {
    if (!adj[k].p)
      adj[k] = make_tensor(e_.arena(), batched_shape(nodes_[k].val.shape(), batch), true, e_.stream());
    return adj[k];
  };
  for (auto& kv : seeds) {
    if (!needs.at(kv.first)) continue;
    Tensor& a = get_adj(kv.first);
    kcheck(axpby(e_.stream(), a.p, kv.second, 1.0, 1.0, a.size()), "seed");
  }
  for (int k = n - 1; k >= 0; --k) {
    if (!adj[k].p || nodes_[k].leaf) continue;
    const Node& nk = nodes_[k];
    for (const Term& tm : nk.terms) {
      DView Cb = out_view(batched_out(tm, batch), adj[k]);
      if (tm.bilinear) {
        const bool na = needs[tm.a.node], nb = needs[tm.b.node];
        if (na) {
          DView Ab = view_of(batched_op(tm.a, batch), get_adj(tm.a.node));
          DView B = view_of(tm.b, nodes_[tm.b.node].val);
          e_.contract(tm.alpha, Cb, B, Ab);
        }
        if (nb) {
          DView Bb = view_of(batched_op(tm.b, batch), get_adj(tm.b.node));
          DView A = view_of(tm.a, nodes_[tm.a.node].val);
          e_.contract(tm.alpha, A, Cb, Bb);
        }
      } else if (needs[tm.a.node]) {
        DView Ab = view_of(batched_op(tm.a, batch), get_adj(tm.a.node));
        e_.linear(tm.alpha, Cb, Ab);
      }
    }
  }
  std::map<int, Tensor> out;
  for (int w : wrt) out[w] = get_adj(w);
  return out;
}

}  // namespace nm
