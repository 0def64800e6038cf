// Device tensor engine with a recording tape.
//
// A Graph is a list of nodes; each node holds one contiguous fp64 device
// tensor equal to a sum of terms, where a term is either
//   * a contraction  alpha * einsum(la, lb -> lout)(A_view, B_view), or
//   * a linear view  alpha * einsum(la -> lout)(A_view)   (permutation,
//     block extraction, diagonal, partial sums),
// written into a sub-box of the node.  Operands are strided views (sub-box +
// index labels, repeated labels = diagonals) of earlier nodes.  Values are
// computed eagerly when a node is created.
//
// Because every node is multilinear in its inputs, derivatives are taken on
// the graph itself:
//   * jvp(): appends one tangent node per node that depends on a seeded leaf
//     (product rule on each contraction term), so tangents can themselves be
//     differentiated;
//   * vjp(): reverse sweep accumulating adjoints into the requested nodes.
// Contractions run as [batch][M][K] x [batch][K][N] GEMMs on the FP64 matrix
// cores after packing the operand views with the strided-view kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.h"

namespace nm {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what);

// Device memory: a stack of chunks with mark/rewind (LIFO lifetimes).
class Arena {
 public:
  ~Arena();
  double* alloc(int64_t ndouble);
  struct Mark { size_t chunk; size_t top; };
  Mark mark() const { return {cur_, chunks_.empty() ? 0 : chunks_[cur_].top}; }
  void rewind(Mark m);
  size_t peak_bytes() const { return peak_; }
  // frees the chunks after the current one (unused since the last rewind)
  void trim();
  size_t reserved_bytes() const;

 private:
  struct Chunk { char* base; size_t cap; size_t top; };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
  size_t peak_ = 0, live_ = 0;
};

struct Range { int64_t lo, len; };

struct Tensor {
  double* p = nullptr;
  int nd = 0;
  int64_t d[kMaxViewDims] = {0};
  // values unchanged when the first and second halves of the indices are
  // swapped (a symmetric matrix of index pairs, e.g. (ac|bd) as [cd][ab])
  bool pair_sym = false;
  // never written after creation (integrals): fp32 packings may be cached
  bool constant = false;
  // unchanged until Engine::clear_frozen() (the recorded values of a
  // linearisation): its low-precision packings are cached until then
  bool frozen = false;
  int64_t size() const {
    int64_t s = 1;
    for (int k = 0; k < nd; ++k) s *= d[k];
    return s;
  }
  std::vector<int64_t> shape() const { return std::vector<int64_t>(d, d + nd); }
};

struct Op {             // operand: node + box + labels (one label per dim)
  int node = -1;
  std::string lab;
  std::vector<Range> box;   // empty = whole tensor
};

struct Term {
  double alpha = 1.0;
  bool bilinear = false;
  Op a, b;                 // b unused for linear terms
  std::string olab;        // labels of the output box dims
  std::vector<Range> obox; // empty = whole node
};

struct Node {
  Tensor val;
  std::vector<Term> terms;  // empty for leaves
  bool leaf = false;
};

// Device view with distinct labels (repeats merged into one strided dim).
struct DView {
  double* p = nullptr;
  int nd = 0;
  bool pair_sym = false;   // see Tensor::pair_sym (whole tensors only)
  bool constant = false;   // view of a Tensor::constant tensor
  bool frozen = false;     // view of a Tensor::frozen tensor
  int64_t dims[kMaxViewDims] = {0};
  int64_t str[kMaxViewDims] = {0};
  char lab[kMaxViewDims] = {0};
};

class Engine {
 public:
  Engine(hipStream_t s);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  hipStream_t stream() const { return s_; }
  Arena& arena() { return arena_; }

  // primitives on views
  // C (+)= alpha A.B ; C (+)= alpha sum A.  overwrite: C = ... (C's old values ignored)
  void contract(double alpha, const DView& A, const DView& B, const DView& C, bool overwrite = false);
  void linear(double alpha, const DView& A, const DView& C, bool overwrite = false);
  double* scratch_reduce();
  double* scalar_slot(int k);   // small device scalars
  uint64_t gemm_flops() const { return flops_; }
  void reset_flops() { flops_ = 0; }
  // Mixed precision: unbatched contractions of at least lowp_min_flops run
  // with fp32 operands on the FP32 matrix cores (fp32 accumulation, fp64
  // result) while set_lowp(true) is in effect.
  void set_lowp(bool on) { lowp_ = on; }
  void set_lowp_min_flops(double f) { lowp_min_flops_ = f; }
  bool lowp() const { return lowp_; }
  uint64_t lowp_flops() const { return lowp_flops_; }
  // With set_bf16(true) as well, those contractions carry each fp32 operand
  // as a bfloat16 pair (hi + lo) and run three bf16 matrix-core products
  // (fp32 accumulation): about 2^-16 relative instead of fp32's 2^-24.
  void set_bf16(bool on) { bf16_ = on; }
  bool bf16() const { return bf16_; }
  // Releases the packings of frozen tensors (their values may change next).
  void clear_frozen();

 private:
  hipStream_t s_;
  Arena arena_;
  double* red_ = nullptr;
  double* scal_ = nullptr;
  uint64_t flops_ = 0;
  bool lowp_ = false;
  double lowp_min_flops_ = 1e9;
  uint64_t lowp_flops_ = 0;
  // fp32 packings of constant operands, keyed by source view and order
  std::map<std::string, float*> f32_cache_;
  size_t f32_cache_bytes_ = 0;
  const float* packed_f32(const DView& src, const std::string& order, bool cache = true);
  // bfloat16 pair of src in `order` as [rows][Kp] (last K elements of each
  // row from the trailing labels, zero-padded to Kp); constants cached
  bool bf16_ = false;
  std::map<std::string, uint16_t*> bf16_cache_;
  size_t bf16_cache_bytes_ = 0;
  // packings of frozen views (fp32 or bf16 pairs), released by clear_frozen()
  std::map<std::string, void*> frozen_cache_;
  size_t frozen_cache_bytes_ = 0;
  void* frozen_lookup(const std::string& key) const;
  void* frozen_store(const std::string& key, size_t bytes);
  void packed_bf16(const DView& src, const std::string& order, int64_t rows, int64_t K, int64_t Kp,
                   const uint16_t** pairs);
};

class Graph {
 public:
  explicit Graph(Engine& e) : e_(e) {}
  ~Graph();
  int leaf(const Tensor& t);
  int node(const std::vector<int64_t>& shape, const std::vector<Term>& terms);
  const Tensor& val(int id) const { return nodes_[id].val; }
  int size() const { return (int)nodes_.size(); }

  // Tangents of every node from `first` on, given tangents of some nodes
  // (node -> tangent node).  Returns the completed map (absent = zero).
  // batch > 0: `batch` directions at once; every tangent node (seeds too)
  // has shape [batch] + the shape of its primal node.
  std::map<int, int> jvp(const std::map<int, int>& seeds, int first = 0, int64_t batch = 0);

  // Reverse sweep.  seeds: node -> device tensor (same shape) holding the
  // adjoint of a scalar functional; returns adjoints of `wrt` nodes (device
  // tensors allocated in the arena; zero-filled when unreachable).
  // batch > 0: `batch` functionals at once, seeds and adjoints of shape
  // [batch] + the node's shape.
  std::map<int, Tensor> vjp(const std::map<int, const double*>& seeds,
                            const std::vector<int>& wrt, int64_t batch = 0);

  // Truncate the tape to `n` nodes (values of removed nodes are released
  // when the arena is rewound by the caller).
  void truncate(int n) { nodes_.resize(n); }
  // Marks the values of nodes [0, n) frozen (Tensor::frozen).
  void freeze(int n) {
    for (int k = 0; k < n && k < (int)nodes_.size(); ++k) nodes_[k].val.frozen = true;
  }
  Engine& engine() { return e_; }
  // strided view of an operand (box + labels) of an existing node
  DView view(const Op& o) const { return view_of(o, nodes_.at(o.node).val); }

 private:
  DView view_of(const Op& op, const Tensor& t) const;
  DView out_view(const Term& tm, const Tensor& t) const;
  Engine& e_;
  std::vector<Node> nodes_;
};

// Term builders.
inline Op op(int node, const std::string& lab, std::vector<Range> box = {}) {
  return Op{node, lab, std::move(box)};
}
inline Term mul(double alpha, Op a, Op b, const std::string& olab, std::vector<Range> obox = {}) {
  Term t;
  t.alpha = alpha;
  t.bilinear = true;
  t.a = std::move(a);
  t.b = std::move(b);
  t.olab = olab;
  t.obox = std::move(obox);
  return t;
}
inline Term lin(double alpha, Op a, const std::string& olab, std::vector<Range> obox = {}) {
  Term t;
  t.alpha = alpha;
  t.bilinear = false;
  t.a = std::move(a);
  t.olab = olab;
  t.obox = std::move(obox);
  return t;
}

// Contiguous tensor helpers.
Tensor make_tensor(Arena& a, const std::vector<int64_t>& shape, bool zero, hipStream_t s);
DView full_view(const Tensor& t, const std::string& lab);

}  // namespace nm
