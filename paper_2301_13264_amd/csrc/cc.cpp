// Closed-shell CCSD derivative couplings on the device: residual graph,
// ground state, EOM (Davidson), multipliers, densities and the coupling
// contraction, behind the C ABI of include/nacme.h.
//
// Only the residual Omega(t; f, g) is written out by hand (the spin-adapted
// T1-transformed CCSD equations).  Every other operator of the Lagrangian is
// obtained by differentiating that graph on the device:
//   A R            = forward derivative (jvp) of Omega along R      (Sec. II B)
//   L^T A          = reverse derivative (vjp) of L.Omega             (Sec. II B)
//   F(gamma) R     = reverse derivative of gamma.(A R)               (Sec. II B)
//   densities      = reverse derivative of the Hamiltonian-linear
//                    part of the Lagrangian w.r.t. the integrals      (Sec. II C)
//   eta_kappa, A^HF = derivatives through H -> exp(kappa) H exp(-kappa),
//                    linearised at kappa = 0                          (Sec. II A/B)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/nacme.h"
#include "engine.h"
#include "linalg.h"

#include <cstdio>
#include <cstdlib>

namespace nm {

static bool verbose() {
  static int v = -1;
  if (v < 0) v = std::getenv("NACME_VERBOSE") ? 1 : 0;
  return v == 1;
}

// ------------------------------------------------------------------ context
// Operand groups of the one-sided two-electron density blocks, by what a
// perturbation direction supplies for the unlifted half of each integral use:
// vo(dB) and oo(dB) (T1-transformed blocks of its factor), their forward
// derivatives along R1_j, and the bare dB_ov block.
enum { G_VO, G_VOT, G_OO, G_OOT, G_OV, NGRP };

// Two-electron density of a Lagrangian, kept as the adjoints of the places
// where the integrals enter it (never as an n^4 tensor): the bare blocks W,
// Wov, Gov and the T1-transformed blocks / Fock correction of the residual
// graph (indexed by Use), plus the Hartree-Fock energy term of the energy
// Lagrangian.  densities() lifts one half of every use onto the packed pairs
// of the factor (gam); the vvvv block stays factorised.
struct PairData {
  double* zeta = nullptr;    // amplitude-shaped
  double* gamma = nullptr;   // amplitude-shaped
  double* eta_t = nullptr;
  double* kbar = nullptr;    // [o][v]
  double* eta_k = nullptr;   // [o][v]
  double* dtrans = nullptr;  // [n][n] transition density
  double* Fbar = nullptr;    // [n][n]  d Phi / d f
  double* Deff = nullptr;    // [n][n]
  // vvvv block d Phi / d W[c][d][a][b] = sum_ij t_ij^cd Y0_ij^ab
  // (+ R_ij^cd Y1_ij^ab, R = R_jr): Y0 (and Y1), the adjoints of the ladder's
  // output in the residual (and in its derivative along R_jr)
  double* ylad = nullptr;    // [nlad][o][o][v][v]
  int nlad = 0, jr = -1;
  double* gWov = nullptr;    // [v][v][o][v]  d Phi / d Wov
  double* gGov = nullptr;    // [o][v][o][v]  d Phi / d Gov
  double* guse[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // adjoints of the same uses in the forward derivative along R_j (the
  // integrals' part of gamma . A R_j), when the pair has a right state
  double* guse_t[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool has_tan = false;
  double* Bbar = nullptr;    // [P][n][n]  d Phi / d B through every use (orbital rotation)
  bool hf_term = false;      // energy Lagrangian: E_HF's two-electron part
  // one-sided blocks [gcols][m]: column group g (offset goff[g], glen[g]
  // operand entries) holds, for each operand entry, the lifted half of the
  // uses as a linear form on the packed symmetric pairs of the factor
  // (m = n (n + 1) / 2, order [oo | ov | vv])
  double* gam = nullptr;
  int64_t goff[NGRP] = {0, 0, 0, 0, 0}, glen[NGRP] = {0, 0, 0, 0, 0}, gcols = 0;
  bool have_mult = false, have_dens = false;
};

}  // namespace nm

struct cc_ctx {
  int o = 0, v = 0, n = 0, naux = 0;
  int64_t N = 0;  // amplitude-shaped length
  cc_opts opts{};
  hipStream_t s = nullptr;
  std::unique_ptr<nm::Engine> eng;
  std::vector<void*> owned;
  nm::Tensor eps, f;
  nm::Tensor B;        // density-fitting factor B[P][p][q], (pq|rs) = sum_P B[P][p][q] B[P][r][s]
  // bare integral blocks: W[c][d][a][b] = (ac|bd), Wov[c][d][k][b] = (kc|bd),
  // Gov[k][c][l][d] = (kc|ld)
  nm::Tensor W, Wov, Gov;
  std::vector<double> eps_h;
  double* t = nullptr;
  bool have_guess = false;
  // starting vectors of the next right / left EOM solve (cc_set_guess), e.g.
  // the states of a neighbouring geometry; used once, then dropped
  std::map<int, double*> guess_R, guess_L;
  int stage = 0;  // 1 ground done
  bool have_right = false, have_left = false, gauged = false;
  double ecorr = 0.0;
  int nroots = 0;
  std::vector<double> omega_r, omega_l, R0;
  std::vector<double*> R, L;
  std::map<std::pair<int, int>, nm::PairData> pairs;
  std::string err;
  bool sticky = false;
  int64_t n_right = 0, n_left = 0, n_residual = 0;
  double* rows_part = nullptr;   // partial sums of multi-row dot products
  // Lambda of the ground-state left state <HF| (1 + Lambda) exp(-T)
  // (A^T Lambda = -eta), solved on first use by a pair (0, j)
  double* Lam = nullptr;
  bool have_lam = false;
};

namespace nm {

using Ctx = cc_ctx;

static double* palloc(Ctx& c, int64_t n) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(-4, "device allocation failed (" + std::to_string(n * 8) + " bytes)");
  }
  c.owned.push_back(p);
  return (double*)p;
}

static void kc(int rc, const char* what) {
  if (rc != 0) throw Error(-3, std::string("kernel launch failed: ") + what);
}

static void sync(Ctx& c) { hip_check(hipStreamSynchronize(c.s), "stream synchronize"); }

static double d2h(Ctx& c, const double* dptr) {
  double x;
  hip_check(hipMemcpyAsync(&x, dptr, sizeof(double), hipMemcpyDeviceToHost, c.s), "memcpy D2H");
  sync(c);
  return x;
}

static void copy_d(Ctx& c, double* dst, const double* src, int64_t n) {
  if (n > 0)
    hip_check(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c.s), "memcpy D2D");
}

// rows k of `len` doubles: dst[k * ldd ...] = src[k * lds ...]
static void copy_rows(Ctx& c, double* dst, int64_t ldd, const double* src, int64_t lds, int64_t len,
                      int64_t rows) {
  if (len <= 0 || rows <= 0) return;
  kc(rows_copy(c.s, dst, ldd, src, lds, len, rows), "row copy");
}

struct ArenaScope {
  Arena& a;
  Arena::Mark m;
  explicit ArenaScope(Arena& ar) : a(ar), m(ar.mark()) {}
  ~ArenaScope() { a.rewind(m); }
};

// Ground state in the mixed modes: fp32-operand residuals until max|Omega|
// falls below kMixedSwitch, then fp64 residuals to the tolerance.
constexpr double kMixedSwitch = 1e-6;
// bf16 mode: bfloat16-pair operands while max|Omega| > kBf16GroundSwitch,
// fp32 operands from there to kMixedSwitch
constexpr double kBf16GroundSwitch = 1e-3;
// Eigen- and linear solvers: fp32-operand images carry about 1e-7 relative
// rounding (bf16 pairs about 1e-5), so the residual norms computed from them
// level off there; at that point (or when they stall) the current solution
// gets fp64 images.
constexpr double kEigSwitch = 1e-7, kEigSwitchBf16 = 1e-5;
static bool mixed(const Ctx& c) {
  return c.opts.precision == CC_FP32_REFINE || c.opts.precision == CC_BF16X3_REFINE;
}
// the solvers' low-precision operator: bf16 pairs in CC_BF16X3_REFINE (the
// ground state keeps fp32 operands: its fp64 phase starts at 1e-5)
static bool solver_bf16(const Ctx& c) { return c.opts.precision == CC_BF16X3_REFINE; }
static double eig_switch(const Ctx& c) { return solver_bf16(c) ? kEigSwitchBf16 : kEigSwitch; }

static Tensor tview(double* p, std::vector<int64_t> shape) {
  Tensor t;
  t.p = p;
  t.nd = (int)shape.size();
  for (int k = 0; k < t.nd; ++k) t.d[k] = shape[k];
  return t;
}

// Vector-space helpers on amplitude-shaped vectors (biorthonormal metric).
static double dot_bio(Ctx& c, const double* x, const double* y) {
  kc(dot(c.s, x, y, c.N, c.o, c.v, 1, c.eng->scratch_reduce(), c.eng->scalar_slot(0)), "dot");
  return d2h(c, c.eng->scalar_slot(0));
}
// Vectors per batched transform: the largest intermediates of a transform
// grow with the batch as a few o v^3 tensors per vector (the tangent and the
// adjoint of the vvov integral use, and their low-precision packings); the
// batch is kept to about 40 GB of them (8 vectors at o = 33, v = 127; 2 at
// v = 250).
static int transform_batch(const Ctx& c) {
  const double per_vec = 4.0 * (double)c.o * c.v * c.v * c.v * 8.0;
  return (int)std::max(1.0, std::min(8.0, std::floor(40e9 / per_vec)));
}

// length of the half layout (singles, doubles (ia) <= (jb)) of an
// amplitude-shaped vector
static int64_t half_len(const Ctx& c) {
  const int64_t nov = (int64_t)c.o * c.v;
  return nov + nov * (nov + 1) / 2;
}
static double dot_plain(Ctx& c, const double* x, const double* y, int64_t n) {
  kc(dot(c.s, x, y, n, 1, 1, 0, c.eng->scratch_reduce(), c.eng->scalar_slot(0)), "dot");
  return d2h(c, c.eng->scalar_slot(0));
}
static double amax(Ctx& c, const double* x, int64_t n) {
  kc(absmax(c.s, x, n, c.eng->scratch_reduce(), c.eng->scalar_slot(1)), "absmax");
  return d2h(c, c.eng->scalar_slot(1));
}
static void axpby_(Ctx& c, double* y, const double* x, double a, double b, int64_t n) {
  kc(axpby(c.s, y, x, a, b, n), "axpby");
}

// h[k] = <V_k, x> for the m rows of V ([m][n] contiguous), in one GEMV and one
// copy to the host; `packed` selects the biorthonormal metric on
// amplitude-shaped vectors.  work: n + m doubles.
static void dots_rows(Ctx& c, const double* V, int m, const double* x, int64_t n, bool packed,
                      double* work, std::vector<double>& h) {
  h.assign(m, 0.0);
  if (m == 0) return;
  const double* xx = x;
  if (packed) {
    kc(apply_metric(c.s, work, x, c.o, c.v, 0), "metric");
    xx = work;
  }
  double* hd = work + n;
  kc(rows_dot(c.s, V, m, n, xx, c.rows_part, hd), "rows_dot");
  hip_check(hipMemcpyAsync(h.data(), hd, m * sizeof(double), hipMemcpyDeviceToHost, c.s), "D2H");
  sync(c);
}

// H[r][k] = <V_k, X_r> for R vectors X [R][n] (rows of V read once per four
// vectors); `packed` selects the biorthonormal metric.  work: R n + R m.
static void dots_rows_multi(Ctx& c, const double* V, int m, const double* X, int R, int64_t n,
                            bool packed, double* work, std::vector<double>& H) {
  H.assign((size_t)R * m, 0.0);
  if (m == 0 || R == 0) return;
  const double* xx = X;
  if (packed) {
    for (int r = 0; r < R; ++r)
      kc(apply_metric(c.s, work + (int64_t)r * n, X + (int64_t)r * n, c.o, c.v, 0), "metric");
    xx = work;
  }
  double* hd = work + (int64_t)R * n;
  for (int r0 = 0; r0 < R; r0 += kMaxRhs) {
    const int rr = std::min(kMaxRhs, R - r0);
    kc(rows_dot_multi(c.s, V, m, n, xx + (int64_t)r0 * n, n, rr, c.rows_part, hd + (int64_t)r0 * m),
       "rows_dot_multi");
  }
  hip_check(hipMemcpyAsync(H.data(), hd, H.size() * sizeof(double), hipMemcpyDeviceToHost, c.s), "D2H");
  sync(c);
}

// X_r -= sum_k H[r][k] V_k for R vectors X [R][n]; hd: R m device doubles.
static void sub_rows_multi(Ctx& c, const double* V, int m, const std::vector<double>& H, double* X,
                           int R, int64_t n, double* hd) {
  if (m == 0 || R == 0) return;
  hip_check(hipMemcpyAsync(hd, H.data(), (size_t)R * m * sizeof(double), hipMemcpyHostToDevice, c.s),
            "H2D");
  for (int r0 = 0; r0 < R; r0 += kMaxRhs) {
    const int rr = std::min(kMaxRhs, R - r0);
    kc(rows_axpy_multi(c.s, V, m, n, hd + (int64_t)r0 * m, -1.0, X + (int64_t)r0 * n, n, rr),
       "rows_axpy_multi");
  }
}

// x -= sum_k h[k] V_k (one GEMM); hd: m device doubles.
static void sub_rows(Ctx& c, const double* V, int m, const std::vector<double>& h, double* x, int64_t n,
                     double* hd) {
  if (m == 0) return;
  hip_check(hipMemcpyAsync(hd, h.data(), m * sizeof(double), hipMemcpyHostToDevice, c.s), "H2D");
  kc(rows_axpy(c.s, V, m, n, hd, -1.0, x), "rows_axpy");
}

// ------------------------------------------------------------ residual graph
// Integral-use nodes of the residual graph: the T1-transformed two-electron
// blocks, each sum_P Bhat_L[P](x) Bhat_R[P] of two blocks of the transformed
// factor, and the Fock correction.  Each is bilinear in the two factor leaves,
// so the adjoint of the node (a block of the transformed two-electron density)
// contracted with the same node built from a direction's factor gives that
// use's part of the coupling.
enum Use { U_VOVO, U_OOOO, U_OOVV, U_VOOV, U_VVOV, U_VVOO, U_OOOV, U_FCORR, NUSE };

struct ResNodes {
  int t1, t2, f, bl, br, w, wov, gov;
  int om1, om2;
  int ev = -1, eo = -1;   // dressed one-particle blocks Ev[b][c], Eo[k][j] of the doubles equations
  int first;  // first non-leaf node of the residual
  int use[NUSE];
};

// Blocks of the T1-transformed factor Bhat[P] = X B[P] Y^T, with X = 1 - t~ on
// creator indices and Y = 1 + t~^T on annihilator indices, t~[a,i] = t_ai (X is
// the identity on occupied creators, Y on virtual annihilators):
//   D[P][p][k]  = sum_c B[P][p][c] t_kc                 (p all, k occupied)
//   Boo[P][k][l] = B[P][k][l] + D[P][k][l]
//   Bvv[P][a][c] = B[P][a][c] - sum_l t_la B[P][l][c]
//   Bvo[P][a][k] = B[P][a][k] + D[P][a][k] - sum_l t_la Boo[P][l][k]
//   Bov[P][k][c] = B[P][k][c]
struct FactorNodes { int d, oo, vv, vo; };
static FactorNodes factor_graph(Graph& G, Ctx& c, int t1, int b, bool with_vv = true) {
  // P: the leaf's leading extent (the auxiliary index, or any batch of
  // factor-shaped matrices)
  const int64_t o = c.o, v = c.v, n = c.n, P = G.val(b).d[0];
  const Range AP{0, P}, A{0, n}, O{0, o}, V{o, v}, Ol{0, o};
  FactorNodes r;
  r.d = G.node({P, n, o}, {mul(1, op(b, "Ppc", {AP, A, V}), op(t1, "kc"), "Ppk")});
  r.oo = G.node({P, o, o}, {lin(1, op(b, "Pkl", {AP, O, O}), "Pkl"),
                            lin(1, op(r.d, "Pkl", {AP, O, Ol}), "Pkl")});
  r.vv = !with_vv ? -1
                   : G.node({P, v, v}, {lin(1, op(b, "Pac", {AP, V, V}), "Pac"),
                                        mul(-1, op(t1, "la"), op(b, "Plc", {AP, O, V}), "Pac")});
  r.vo = G.node({P, v, o}, {lin(1, op(b, "Pak", {AP, V, O}), "Pak"),
                            lin(1, op(r.d, "Pak", {AP, V, Ol}), "Pak"),
                            mul(-1, op(t1, "la"), op(r.oo, "Plk"), "Pak")});
  return r;
}

// Operands of the T1-transformed two-electron use u (< U_FCORR): the block
// sum_P a[P] (x) b[P] with output labels `out` (L, R: the transformed blocks
// of the two factor leaves; br: the right factor leaf itself).
struct UseSpec { Op a, b; std::string out; std::vector<int64_t> shape; };
static UseSpec use_spec(Ctx& c, int u, const FactorNodes& L, const FactorNodes& R, int br) {
  const int64_t o = c.o, v = c.v, P = c.naux;
  const Range AP{0, P}, O{0, o}, V{o, v};
  switch (u) {
    case U_VOVO: return {op(L.vo, "Pai"), op(R.vo, "Pbj"), "aibj", {v, o, v, o}};
    case U_OOOO: return {op(L.oo, "Pki"), op(R.oo, "Plj"), "kilj", {o, o, o, o}};
    case U_OOVV: return {op(L.oo, "Pki"), op(R.vv, "Pac"), "kiac", {o, o, v, v}};
    case U_VOOV: return {op(L.vo, "Pai"), op(br, "Pkc", {AP, O, V}), "aikc", {v, o, o, v}};
    case U_VVOV: return {op(L.vv, "Pad"), op(br, "Pkc", {AP, O, V}), "adkc", {v, v, o, v}};
    case U_VVOO: return {op(L.vv, "Pac"), op(R.oo, "Pki"), "acki", {v, v, o, o}};
    default: return {op(L.oo, "Pki"), op(br, "Plc", {AP, O, V}), "kilc", {o, o, o, v}};
  }
}

// Omega(t; f, g) of closed-shell CCSD in the T1-transformed form with
// density-fitted integrals g_pqrs = sum_P B[P][p][q] B[P][r][s] (Mulliken).
// The transformed integrals are ghat_pqrs = sum_P Bhat[P][p][q] Bhat[P][r][s];
// the two factors of every product are separate leaves (bl, br) that hold the
// same values, so that the graph is linear in each.  The transformed blocks
// the equations use are built as GEMMs over P from the factor blocks above.
// The vvvv block only enters the particle-particle ladder; that term is
// evaluated on the bare integrals W[cd][ab] = (ac|bd) with the creator
// transforms written out:
//   sum_cd t_ij^cd ghat_acbd = sum_cd t_ij^cd g_acbd - sum_k t_ak Y1_ijkb
//       - sum_l t_bl Y1_jila + sum_kl t_ak t_bl Z_ijkl,
//   Y1_ijkb = sum_cd t_ij^cd g_kcbd,  Z_ijkl = sum_cd t_ij^cd g_kcld,
// so that derivatives of the residual contain one ladder GEMM, not two
// (W, Wov[c][d][k][b] = (kc|bd) and Gov[k][c][l][d] = (kc|ld) are bare leaves).
// The transformed Fock matrix is Fhat = X (f + 2 J(t1) - K(t1)) Y^T, where
// J(t1) - J = 2 sum_P (sum_k D[P][k][k]) B[P] and K(t1) - K =
// sum_P D[P] B[P][occ rows]; the singles and doubles projections are those
// of the oracle's residual.
static ResNodes residual_graph(Graph& G, Ctx& c, const Tensor& T1, const Tensor& T2,
                               const Tensor& F, const Tensor& Bf, const Tensor& Wt,
                               const Tensor& Wov, const Tensor& Gov) {
  const int64_t o = c.o, v = c.v, n = c.n, P = c.naux;
  const Range O{0, o}, V{o, v}, A{0, n}, AP{0, P}, Ol{0, o};
  ResNodes r;
  r.t1 = G.leaf(T1);
  r.t2 = G.leaf(T2);
  r.f = G.leaf(F);
  r.bl = G.leaf(Bf);
  r.br = G.leaf(Bf);
  r.w = G.leaf(Wt);
  r.wov = G.leaf(Wov);
  r.gov = G.leaf(Gov);
  r.first = G.size();
  const int t1 = r.t1, t2 = r.t2, f = r.f;
  const FactorNodes L = factor_graph(G, c, t1, r.bl), R = factor_graph(G, c, t1, r.br);
  // transformed two-electron blocks (integral uses)
  for (int u = 0; u < U_FCORR; ++u) {
    const UseSpec us = use_spec(c, u, L, R, r.br);
    r.use[u] = G.node(us.shape, {mul(1, us.a, us.b, us.out)});
  }
  const int gvovo = r.use[U_VOVO], goooo = r.use[U_OOOO], goovv = r.use[U_OOVV],
            gvoov = r.use[U_VOOV], gvvov = r.use[U_VVOV], gvvoo = r.use[U_VVOO],
            gooov = r.use[U_OOOV];
  // Fock correction 2 (J(t1) - J) - (K(t1) - K)
  const int trd = G.node({P}, {lin(1, op(L.d, "Pkk", {AP, O, Ol}), "P")});
  const int fcorr = G.node({n, n}, {mul(2, op(trd, "P"), op(r.br, "Ppq"), "pq"),
                                    mul(-1, op(L.d, "Ppk"), op(r.br, "Pkq", {AP, O, A}), "pq")});
  r.use[U_FCORR] = fcorr;
  const Op g_ovov = op(r.gov, "kcld");
  // transformed Fock matrix
  const int fp = G.node({n, n}, {lin(1, op(f, "pq"), "pq"), lin(1, op(fcorr, "pq"), "pq")});
  const int f1 = G.node({n, n}, {lin(1, op(fp, "pq"), "pq"),
                                 mul(-1, op(t1, "ka"), op(fp, "kq", {O, A}), "aq", {V, A})});
  const int Fh = G.node({n, n}, {lin(1, op(f1, "pq"), "pq"),
                                 mul(1, op(f1, "pc", {A, V}), op(t1, "qc"), "pq", {A, O})});
  const int u = G.node({o, o, v, v}, {lin(2, op(t2, "ijab"), "ijab"), lin(-1, op(t2, "ijba"), "ijab")});
  // singles
  r.om1 = G.node({o, v}, {mul(1, op(u, "kicd"), op(gvvov, "adkc"), "ia"),
                          mul(-1, op(u, "klac"), op(gooov, "kilc"), "ia"),
                          mul(1, op(u, "ikac"), op(Fh, "kc", {O, V}), "ia"),
                          lin(1, op(Fh, "ai", {V, O}), "ia")});
  // ladder pieces on bare integrals
  const int Y1 = G.node({o, o, o, v}, {mul(1, op(t2, "ijcd"), op(r.wov, "cdkb"), "ijkb")});
  const int Z = G.node({o, o, o, o}, {mul(1, op(t2, "ijcd"), g_ovov, "ijkl")});
  const int Zt = G.node({o, o, v, o}, {mul(1, op(t1, "ka"), op(Z, "ijkl"), "ijal")});
  // doubles
  const int W = G.node({o, o, o, o}, {lin(1, op(goooo, "kilj"), "kilj"),
                                      mul(1, op(t2, "ijcd"), g_ovov, "kilj")});
  const int Xc = G.node({o, o, v, v}, {lin(1, op(goovv, "kiac"), "kiac"),
                                       mul(-0.5, op(t2, "liad"), op(r.gov, "kdlc"), "kiac")});
  const int Lvoov = G.node({v, o, o, v}, {lin(2, op(gvoov, "aikc"), "aikc"),
                                          lin(-1, op(gvvoo, "acki"), "aikc")});
  const int Lovov = G.node({o, v, o, v}, {lin(2, op(r.gov, "ldkc"), "ldkc"),
                                          lin(-1, op(r.gov, "lckd"), "ldkc")});
  const int Xd = G.node({v, o, o, v}, {lin(1, op(Lvoov, "aikc"), "aikc"),
                                       mul(0.5, op(u, "ilad"), op(Lovov, "ldkc"), "aikc")});
  const int Ev = G.node({v, v}, {lin(1, op(Fh, "bc", {V, V}), "bc"),
                                 mul(-1, op(u, "klbd"), op(r.gov, "ldkc"), "bc")});
  const int Eo = G.node({o, o}, {lin(1, op(Fh, "kj", {O, O}), "kj"),
                                 mul(1, op(u, "ljcd"), op(r.gov, "kdlc"), "kj")});
  r.ev = Ev;
  r.eo = Eo;
  // Q_ijab = sum_kc t_kjbc Xc_kiac; the exchange partner sum_kc t_kibc Xc_kjac
  // is Q with i and j swapped, added as a permutation instead of a second GEMM
  const int Q = G.node({o, o, v, v}, {mul(1, op(t2, "kjbc"), op(Xc, "kiac"), "ijab")});
  const int Pn = G.node({o, o, v, v}, {lin(-0.5, op(Q, "ijab"), "ijab"),
                                       lin(-1, op(Q, "jiab"), "ijab"),
                                       mul(0.5, op(u, "jkbc"), op(Xd, "aikc"), "ijab"),
                                       mul(1, op(t2, "ijac"), op(Ev, "bc"), "ijab"),
                                       mul(-1, op(t2, "ikab"), op(Eo, "kj"), "ijab")});
  r.om2 = G.node({o, o, v, v}, {mul(1, op(t2, "ijcd"), op(r.w, "cdab"), "ijab"),
                                lin(1, op(gvovo, "aibj"), "ijab"),
                                mul(-1, op(t1, "ka"), op(Y1, "ijkb"), "ijab"),
                                mul(-1, op(Y1, "jila"), op(t1, "lb"), "ijab"),
                                mul(1, op(Zt, "ijal"), op(t1, "lb"), "ijab"),
                                mul(1, op(t2, "klab"), op(W, "kilj"), "ijab"),
                                lin(1, op(Pn, "ijab"), "ijab"),
                                lin(1, op(Pn, "jiba"), "ijab")});
  return r;
}

// E_corr = 2 sum f_ia t_ai + sum (t_aibj + t_ai t_bj)(2 g_iajb - g_ibja).
struct EnergyNodes { int t1, t2, f, gov, e; };
static EnergyNodes energy_graph(Graph& G, Ctx& c, const Tensor& T1, const Tensor& T2) {
  const int64_t o = c.o, v = c.v;
  const Range O{0, o}, V{o, v};
  EnergyNodes r;
  r.t1 = G.leaf(T1);
  r.t2 = G.leaf(T2);
  const int f = G.leaf(c.f), g = G.leaf(c.Gov);
  r.f = f;
  r.gov = g;
  const int tau = G.node({o, o, v, v}, {lin(1, op(r.t2, "ijab"), "ijab"),
                                        mul(1, op(r.t1, "ia"), op(r.t1, "jb"), "ijab")});
  const int Lb = G.node({o, v, o, v}, {lin(2, op(g, "iajb"), "iajb"),
                                       lin(-1, op(g, "ibja"), "iajb")});
  r.e = G.node({}, {mul(2, op(f, "ia", {O, V}), op(r.t1, "ia"), ""),
                    mul(1, op(tau, "ijab"), op(Lb, "iajb"), "")});
  return r;
}

static Tensor T1of(Ctx& c, double* x) { return tview(x, {c.o, c.v}); }
static Tensor T2of(Ctx& c, double* x) {
  return tview(x + (int64_t)c.o * c.v, {c.o, c.o, c.v, c.v});
}

// Residual at amplitudes x -> out (amplitude-shaped).
// dressed orbital energies deps[n]: the diagonals of Eo (occupied) and Ev
// (virtual), the one-particle blocks of the doubles equations
static void dressed_diagonal(Ctx& c, Graph& G, const ResNodes& r, double* deps) {
  ViewSpec vo;
  vo.nd = 1;
  vo.dims[0] = c.o;
  vo.istr[0] = c.o + 1;
  vo.ostr[0] = 1;
  kc(view_gather(c.s, deps, G.val(r.eo).p, vo, 1.0, 0.0), "dressed diagonal");
  ViewSpec vv;
  vv.nd = 1;
  vv.dims[0] = c.v;
  vv.istr[0] = c.v + 1;
  vv.ostr[0] = 1;
  vv.obase = c.o;
  kc(view_gather(c.s, deps, G.val(r.ev).p, vv, 1.0, 0.0), "dressed diagonal");
}

// out = Omega(x); deps (optional) <- the dressed orbital energies at x
static void residual(Ctx& c, double* x, double* out, double* deps = nullptr) {
  ++c.n_residual;
  ArenaScope sc(c.eng->arena());
  Graph G(*c.eng);
  ResNodes r = residual_graph(G, c, T1of(c, x), T2of(c, x), c.f, c.B, c.W, c.Wov, c.Gov);
  const int64_t nov = (int64_t)c.o * c.v;
  copy_d(c, out, G.val(r.om1).p, nov);
  copy_d(c, out + nov, G.val(r.om2).p, c.N - nov);
  if (deps) dressed_diagonal(c, G, r, deps);
}

static double energy(Ctx& c, double* x) {
  ArenaScope sc(c.eng->arena());
  Graph G(*c.eng);
  EnergyNodes e = energy_graph(G, c, T1of(c, x), T2of(c, x));
  return d2h(c, G.val(e.e).p);
}

// dE/dt . R (full-tensor directional derivative).
static double energy_jvp(Ctx& c, double* x, double* Rv) {
  ArenaScope sc(c.eng->arena());
  Graph G(*c.eng);
  EnergyNodes e = energy_graph(G, c, T1of(c, x), T2of(c, x));
  const int r1 = G.leaf(T1of(c, Rv)), r2 = G.leaf(T2of(c, Rv));
  auto tan = G.jvp({{e.t1, r1}, {e.t2, r2}});
  if (!tan.count(e.e)) return 0.0;
  return d2h(c, G.val(tan[e.e]).p);
}

// --------------------------------------------------- linearisation (tape)
// The residual graph recorded at the current amplitudes; right and left
// Jacobian transforms reuse it for every trial vector.
struct Tape {
  Ctx& c;
  Arena::Mark base;
  Graph G;
  ResNodes r;
  explicit Tape(Ctx& cc) : c(cc), base(cc.eng->arena().mark()), G(*cc.eng) {
    // the recorded primal values are always fp64; only the derivative sweeps
    // may run with low-precision operands
    const bool lp = c.eng->lowp();
    c.eng->set_lowp(false);
    r = residual_graph(G, c, T1of(c, c.t), T2of(c, c.t), c.f, c.B, c.W, c.Wov, c.Gov);
    c.eng->set_lowp(lp);
    // the recorded values stay as they are while the tape lives: every
    // transform reuses their low-precision packings
    G.freeze(G.size());
    // the solvers' preconditioner: dressed orbital energies at t
    deps = cc.eng->arena().alloc(cc.n);
    dressed_diagonal(cc, G, r, deps);
  }
  double* deps = nullptr;   // [n] dressed orbital energies (Eo_ii, then Ev_aa)
  ~Tape() {
    c.eng->clear_frozen();
    c.eng->arena().rewind(base);
  }

  // y = A x
  void right(const double* x, double* y) {
    ++c.n_right;
    const int n0 = G.size();
    Arena::Mark mk = c.eng->arena().mark();
    const int r1 = G.leaf(T1of(c, const_cast<double*>(x))), r2 = G.leaf(T2of(c, const_cast<double*>(x)));
    auto tan = G.jvp({{r.t1, r1}, {r.t2, r2}}, r.first);
    const int64_t nov = (int64_t)c.o * c.v;
    copy_d(c, y, G.val(tan.at(r.om1)).p, nov);
    copy_d(c, y + nov, G.val(tan.at(r.om2)).p, c.N - nov);
    G.truncate(n0);
    c.eng->arena().rewind(mk);
  }

  // Y[k] = A X[k] for k vectors stored [k][N], in one pass of the graph with
  // a batch index on every tangent (shared primal operands, k-fold GEMMs).
  void right_block(const double* X, double* Y, int k) {
    if (k == 1) return right(X, Y);
    c.n_right += k;
    const int n0 = G.size();
    Arena::Mark mk = c.eng->arena().mark();
    const int64_t nov = (int64_t)c.o * c.v, nd = c.N - nov;
    Tensor b1 = make_tensor(c.eng->arena(), {k, c.o, c.v}, false, c.s);
    Tensor b2 = make_tensor(c.eng->arena(), {k, c.o, c.o, c.v, c.v}, false, c.s);
    copy_rows(c, b1.p, nov, X, c.N, nov, k);
    copy_rows(c, b2.p, nd, X + nov, c.N, nd, k);
    const int r1 = G.leaf(b1), r2 = G.leaf(b2);
    auto tan = G.jvp({{r.t1, r1}, {r.t2, r2}}, r.first, k);
    copy_rows(c, Y, c.N, G.val(tan.at(r.om1)).p, nov, nov, k);
    copy_rows(c, Y + nov, c.N, G.val(tan.at(r.om2)).p, nd, nd, k);
    G.truncate(n0);
    c.eng->arena().rewind(mk);
  }

  // Y[k] = X[k]^T A for k vectors stored [k][N] (one reverse sweep).
  void left_block(const double* X, double* Y, int k) {
    if (k == 1) return left(X, Y);
    c.n_left += k;
    Arena::Mark mk = c.eng->arena().mark();
    const int64_t nov = (int64_t)c.o * c.v, nd = c.N - nov;
    double* tmp = c.eng->arena().alloc(c.N);
    double* s1 = c.eng->arena().alloc((int64_t)k * nov);
    double* s2 = c.eng->arena().alloc((int64_t)k * nd);
    for (int z = 0; z < k; ++z) {
      kc(apply_metric(c.s, tmp, X + (int64_t)z * c.N, c.o, c.v, 0), "metric");
      copy_d(c, s1 + z * nov, tmp, nov);
      copy_d(c, s2 + z * nd, tmp + nov, nd);
    }
    auto adj = G.vjp({{r.om1, s1}, {r.om2, s2}}, {r.t1, r.t2}, k);
    for (int z = 0; z < k; ++z) {
      copy_d(c, tmp, adj[r.t1].p + z * nov, nov);
      copy_d(c, tmp + nov, adj[r.t2].p + z * nd, nd);
      kc(apply_metric(c.s, Y + (int64_t)z * c.N, tmp, c.o, c.v, 1), "metric");
    }
    c.eng->arena().rewind(mk);
  }

  // y = x^T A (packed-gradient convention, amplitude-shaped)
  void left(const double* x, double* y) {
    ++c.n_left;
    Arena::Mark mk = c.eng->arena().mark();
    double* seed = c.eng->arena().alloc(c.N);
    kc(apply_metric(c.s, seed, x, c.o, c.v, 0), "metric");
    const int64_t nov = (int64_t)c.o * c.v;
    auto adj = G.vjp({{r.om1, seed}, {r.om2, seed + nov}}, {r.t1, r.t2});
    double* tmp = c.eng->arena().alloc(c.N);
    copy_d(c, tmp, adj[r.t1].p, nov);
    copy_d(c, tmp + nov, adj[r.t2].p, c.N - nov);
    kc(apply_metric(c.s, y, tmp, c.o, c.v, 1), "metric");
    c.eng->arena().rewind(mk);
  }
};

// ------------------------------------------------------------ ground state
static int ground(Ctx& c, double* e_out, int* it_out) {
  const int64_t N = c.N;
  if (!c.have_guess) kc(fill(c.s, c.t, 0.0, N), "fill");
  ArenaScope sc(c.eng->arena());
  const int m = std::max(1, c.opts.diis_dim);
  double* r = c.eng->arena().alloc(N);
  double* dt = c.eng->arena().alloc(N);
  double* hv = c.eng->arena().alloc((int64_t)m * N);
  double* he = c.eng->arena().alloc((int64_t)m * N);
  std::vector<std::vector<double>> B;   // error overlaps (host)
  int nh = 0, head = 0;
  std::vector<int> slot;                // history order -> slot
  // quasi-Newton step -Omega / D with D from the dressed orbital energies of
  // the current amplitudes (the bare ones at t = 0)
  double* deps = c.eng->arena().alloc(c.n);
  int it = 0;
  double err = 0.0;
  int status = CC_NOT_CONVERGED;
  bool lowp = mixed(c);
  bool bf = lowp && solver_bf16(c);
  c.eng->set_lowp(lowp);
  c.eng->set_bf16(bf);
  for (it = 1; it <= c.opts.maxit; ++it) {
    residual(c, c.t, r, deps);
    err = amax(c, r, N);
    if (!std::isfinite(err)) throw Error(-5, "non-finite CCSD residual");
    if (verbose()) std::fprintf(stderr, "[ground] it %d max|Omega| %.3e\n", it, err);
    if (bf && err < kBf16GroundSwitch) {
      bf = false;
      c.eng->set_bf16(false);
    }
    if (lowp && err < kMixedSwitch) {
      // iterative refinement: the remaining iterations use fp64 residuals
      lowp = false;
      c.eng->set_lowp(false);
      continue;
    }
    if (!lowp && err < c.opts.tol_ground) {
      status = CC_OK;
      break;
    }
    kc(apply_denominator(c.s, dt, r, deps, c.o, c.v, 0.0, 0), "denominator");  // -r/D
    axpby_(c, c.t, dt, 1.0, 1.0, N);
    // DIIS on (t, dt)
    int sidx;
    if (nh < m) {
      sidx = nh++;
      slot.push_back(sidx);
    } else {
      sidx = slot[head];
      slot.erase(slot.begin() + head);
      slot.push_back(sidx);
    }
    copy_d(c, hv + (int64_t)sidx * N, c.t, N);
    copy_d(c, he + (int64_t)sidx * N, dt, N);
    B.resize(m, std::vector<double>(m, 0.0));
    for (int k = 0; k < nh; ++k) {
      const int sk = slot[k];
      const double b = dot_plain(c, he + (int64_t)sidx * N, he + (int64_t)sk * N, N);
      B[sidx][sk] = B[sk][sidx] = b;
    }
    if (nh >= 2) {
      const int q = nh + 1;
      std::vector<double> Am(q * q, 0.0), rhs(q, 0.0);
      double scale = 0.0;
      for (int a = 0; a < nh; ++a) scale = std::max(scale, B[slot[a]][slot[a]]);
      for (int a = 0; a < nh; ++a) {
        for (int b = 0; b < nh; ++b) Am[a * q + b] = B[slot[a]][slot[b]] / scale;
        Am[a * q + nh] = Am[nh * q + a] = -1.0;
      }
      rhs[nh] = -1.0;
      if (lu_solve(Am, rhs, q, 1)) {
        kc(fill(c.s, c.t, 0.0, N), "fill");
        for (int a = 0; a < nh; ++a) axpby_(c, c.t, hv + (int64_t)slot[a] * N, rhs[a], 1.0, N);
      }
    }
  }
  c.eng->set_lowp(false);
  c.eng->set_bf16(false);
  if (it > c.opts.maxit) it = c.opts.maxit;
  c.ecorr = energy(c, c.t);
  if (e_out) *e_out = c.ecorr;
  if (it_out) *it_out = it;
  return status;
}

// ------------------------------------------------------------------ Davidson
struct Ritz {
  std::vector<double> w;
  std::vector<double*> X;  // arena buffers (caller copies)
  int iters = 0;
  bool converged = false;
  bool complex_root = false;
};

// Lowest-nroots eigenpairs of a non-symmetric operator on amplitude-shaped
// vectors (biorthonormal metric), preconditioned by orbital-energy differences
// (peps: the bare orbital energies by default; the EOM solvers pass the
// dressed ones of the linearisation, the diagonals of the one-particle blocks
// of the doubles equations at the converged amplitudes).
// T(X, Y, k) applies the operator to k vectors stored [k][N] at once.
static Ritz davidson(Ctx& c, int nroots, const std::function<void(const double*, double*, int)>& T,
                     std::vector<double*>& out, const std::vector<double*>* guess = nullptr,
                     const double* peps = nullptr) {
  // orbital energies of the preconditioner's denominators
  if (!peps) peps = c.eps.p;
  // Every subspace vector (basis, images, Ritz vectors, corrections) is kept
  // in the half layout (singles and the doubles (ia) <= (jb)), where the
  // biorthonormal product is the plain dot product: half the bytes of every
  // pass over the subspace.  Vectors go to the full symmetric layout only
  // for the transform (and for the caller).
  const int64_t N = half_len(c), nov = (int64_t)c.o * c.v;
  const int nb = nroots + std::max(0, c.opts.davidson_block);
  const int maxm = std::min(kMaxRows, std::max(c.opts.davidson_max, 2 * nb + 2));
  Arena& ar = c.eng->arena();
  ArenaScope sc(ar);
  double* Fin = ar.alloc((int64_t)nb * c.N);   // full-layout transform inputs / outputs
  double* Fout = ar.alloc((int64_t)nb * c.N);
  // T on r half-layout rows: unpack, transform, pack
  const int kt = std::min(nb, transform_batch(c));
  auto Th = [&](const double* Xh, double* Yh, int r) {
    for (int z0 = 0; z0 < r; z0 += kt) {
      const int rr = std::min(kt, r - z0);
      for (int z = 0; z < rr; ++z)
        kc(half_unpack(c.s, Fin + (int64_t)z * c.N, Xh + (int64_t)(z0 + z) * N, c.o, c.v), "unpack");
      T(Fin, Fout, rr);
      for (int z = 0; z < rr; ++z)
        kc(half_pack(c.s, Yh + (int64_t)(z0 + z) * N, Fout + (int64_t)z * c.N, c.o, c.v), "pack");
    }
  };
  auto dotb = [&](const double* x, const double* y) { return dot_plain(c, x, y, N); };
  double* V = ar.alloc((int64_t)maxm * N);
  double* W = ar.alloc((int64_t)maxm * N);
  double* X = ar.alloc((int64_t)nb * N);
  double* AX = ar.alloc((int64_t)nb * N);
  double* Rs = ar.alloc(N);
  double* ydev = ar.alloc((int64_t)nb * maxm);
  std::vector<double> G((size_t)maxm * maxm, 0.0);
  double* work = ar.alloc(N + 2 * maxm);
  double* hd = work + N + maxm;
  // block buffers: corrections [nb][N], metric work and projections
  double* Cblk = ar.alloc((int64_t)nb * N);
  double* workm = ar.alloc((int64_t)nb * N + (int64_t)nb * maxm);
  double* hdm = ar.alloc((int64_t)nb * maxm);
  std::vector<double> h, H;
  int m = 0;
  const bool lowp = mixed(c);
  c.eng->set_lowp(lowp);
  c.eng->set_bf16(lowp && solver_bf16(c));
  // mixed precision: fp64 images of the wanted Ritz vectors, coefficients Z
  double* AXd = lowp ? ar.alloc((int64_t)nroots * N) : nullptr;
  double* zdev = lowp ? ar.alloc((int64_t)nroots * maxm) : nullptr;

  // biorthonormal Gram-Schmidt of x against the basis (two passes, block
  // GEMVs), stored as basis row m (its image, when given, as W row m);
  // false if x is in the span.  Rows without an image get one from flush().
  auto orth = [&](double* x, double* ax) -> bool {
    if (m >= maxm) return false;
    double n0 = std::sqrt(std::max(0.0, dotb(x, x)));
    if (!(n0 > 0)) return false;
    for (int pass = 0; pass < 2 && m > 0; ++pass) {
      dots_rows(c, V, m, x, N, false, work, h);
      sub_rows(c, V, m, h, x, N, hd);
      if (ax) sub_rows(c, W, m, h, ax, N, hd);
    }
    const double n1 = std::sqrt(std::max(0.0, dotb(x, x)));
    if (n1 < 1e-4 * n0 || n1 < 1e-14) return false;
    axpby_(c, V + (int64_t)m * N, x, 1.0 / n1, 0.0, N);
    if (ax) axpby_(c, W + (int64_t)m * N, ax, 1.0 / n1, 0.0, N);
    ++m;
    return true;
  };
  // images of basis rows [m0, m) that have none, in one block application,
  // then the new rows and columns of the projected matrix G = V^T A V
  double t_apply = 0.0;
  auto flush = [&](int m0, int mimg) {
    if (mimg < m) {
      const auto t0 = std::chrono::steady_clock::now();
      Th(V + (int64_t)mimg * N, W + (int64_t)mimg * N, m - mimg);
      if (verbose()) {
        sync(c);
        t_apply += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      }
    }
    const int r = m - m0;
    if (r <= 0) return;
    // columns G[k][j] = <V_k, W_j> and rows G[j][k] = <W_k, V_j>, j >= m0
    dots_rows_multi(c, V, m, W + (int64_t)m0 * N, r, N, false, workm, H);
    for (int jj = 0; jj < r; ++jj)
      for (int k = 0; k < m; ++k) G[(size_t)k * maxm + m0 + jj] = H[(size_t)jj * m + k];
    dots_rows_multi(c, W, m, V + (int64_t)m0 * N, r, N, false, workm, H);
    for (int jj = 0; jj < r; ++jj)
      for (int k = 0; k < m; ++k) G[(size_t)(m0 + jj) * maxm + k] = H[(size_t)jj * m + k];
  };

  // initial guess: given vectors (e.g. the right states for the left
  // problem), then singles unit vectors at the smallest e_a - e_i
  if (guess)
    for (double* gv : *guess) {
      if (m >= nb) break;
      // symmetric part of the given vector, in the half layout
      copy_d(c, Fin, gv, c.N);
      kc(apply_metric(c.s, Fin, Fin, c.o, c.v, 2), "symmetrise");
      kc(half_pack(c.s, Rs, Fin, c.o, c.v), "pack");
      orth(Rs, nullptr);
    }
  if (m < nb) {
    // (the preconditioner's orbital energies decide which singles come first)
    std::vector<double> eh(c.n);
    hip_check(hipMemcpyAsync(eh.data(), peps, c.n * sizeof(double), hipMemcpyDeviceToHost, c.s), "D2H");
    sync(c);
    std::vector<std::pair<double, int64_t>> d;
    for (int i = 0; i < c.o; ++i)
      for (int a = 0; a < c.v; ++a) d.push_back({eh[c.o + a] - eh[i], (int64_t)i * c.v + a});
    std::sort(d.begin(), d.end());
    const double one = 1.0;
    for (int k = 0; k < (int)d.size() && m < nb; ++k) {
      kc(fill(c.s, Rs, 0.0, N), "fill");   // a singles unit vector (same offset in both layouts)
      hip_check(hipMemcpyAsync(Rs + d[k].second, &one, sizeof(double), hipMemcpyHostToDevice, c.s), "H2D");
      sync(c);
      orth(Rs, nullptr);
    }
  }
  flush(0, 0);
  // Mixed precision: every basis image comes from the fp32-operand operator.
  // When the residuals reach the fp32 rounding floor (kEigSwitch or a stall),
  // and again before convergence is accepted, the wanted Ritz vectors
  // X = Y V get fp64 images AXd and their true residual norms are measured.
  // The basis images are then corrected by a rank-nroots update,
  //   W <- W + Z^T D,  D = AXd - Y W,  Z = (Y Y^T)^-1 Y  (so Z Y^T = I),
  // which makes the images of those Ritz vectors exact and leaves the other
  // directions of the basis as they were, and G = V^T W gets the same update.
  // The subspace is kept; later corrections are again imaged in fp32, and
  // their rounding enters the residual only through coefficients of the size
  // of the residual at the update, far below the tolerance.  Only a true
  // (fp64) residual below the tolerance ends the solve.
  double best_lowp = 1e300;
  int stall = 0;
  bool refreshed = false;
  Ritz res;
  double* tmpx = nullptr;   // restart buffers, allocated on the first restart
  double* tmpa = nullptr;
  auto refresh = [&](const std::vector<double>& Y, int nk) -> double {
    c.eng->set_lowp(false);
    Th(X, AXd, nroots);
    c.eng->set_lowp(true);
    double wt = 0.0;
    for (int k = 0; k < nroots; ++k) {
      double* xk = X + (int64_t)k * N;
      double* dk = AXd + (int64_t)k * N;
      copy_d(c, Rs, dk, N);
      axpby_(c, Rs, xk, -res.w[k], 1.0, N);
      const double xn = std::sqrt(dotb(xk, xk));
      wt = std::max(wt, std::sqrt(std::max(0.0, dotb(Rs, Rs))) / xn);
      axpby_(c, dk, AX + (int64_t)k * N, -1.0, 1.0, N);   // D_k
    }
    (void)nk;
    std::vector<double> S((size_t)nroots * nroots, 0.0), Z(Y.begin(), Y.begin() + (size_t)nroots * m);
    for (int a = 0; a < nroots; ++a)
      for (int b = 0; b < nroots; ++b)
        for (int i = 0; i < m; ++i) S[(size_t)a * nroots + b] += Y[(size_t)a * m + i] * Y[(size_t)b * m + i];
    if (!lu_solve(S, Z, nroots, m)) throw Error(-5, "singular Ritz coefficient matrix");
    hip_check(hipMemcpyAsync(zdev, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice, c.s), "H2D");
    kc(gemm_f64(c.s, true, false, m, (int)N, nroots, 1, 1.0, zdev, m, 0, AXd, N, 0, 1.0, W, N, 0),
       "image update");
    dots_rows_multi(c, V, m, AXd, nroots, N, false, workm, H);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        double acc = 0.0;
        for (int k = 0; k < nroots; ++k) acc += H[(size_t)k * m + a] * Z[(size_t)k * m + b];
        G[(size_t)a * maxm + b] += acc;
      }
    return wt;
  };
  // verbose: device time per phase (subspace eigensolve, Ritz vectors,
  // residuals, corrections and their orthogonalisation, projections)
  double t_ph[5] = {0, 0, 0, 0, 0};
  auto t_last = std::chrono::steady_clock::now();
  auto phase = [&](int k) {
    if (!verbose()) return;
    sync(c);
    const auto now = std::chrono::steady_clock::now();
    t_ph[k] += std::chrono::duration<double>(now - t_last).count();
    t_last = now;
  };
  for (int it = 1; it <= c.opts.maxit; ++it) {
    res.iters = it;
    phase(4);
    std::vector<double> Gm((size_t)m * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) Gm[(size_t)a * m + b] = G[(size_t)a * maxm + b];
    std::vector<std::complex<double>> w, Vc;
    if (!eig_nonsym(Gm, m, w, Vc)) throw Error(-5, "subspace eigensolver failed");
    phase(0);
    std::vector<int> ord(m);
    for (int k = 0; k < m; ++k) ord[k] = k;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a].real() < w[b].real(); });
    const int nk = std::min(nb, m);
    std::vector<double> Y((size_t)nk * m);
    res.w.assign(nk, 0.0);
    res.complex_root = false;
    for (int k = 0; k < nk; ++k) {
      const int kk = ord[k];
      res.w[k] = w[kk].real();
      if (k < nroots && std::fabs(w[kk].imag()) > 1e-8 * std::max(1.0, std::fabs(w[kk].real())))
        res.complex_root = true;
      int imax = 0;
      for (int i = 1; i < m; ++i)
        if (std::abs(Vc[(size_t)kk * m + i]) > std::abs(Vc[(size_t)kk * m + imax])) imax = i;
      const std::complex<double> ph = std::conj(Vc[(size_t)kk * m + imax]) / std::abs(Vc[(size_t)kk * m + imax]);
      for (int i = 0; i < m; ++i) Y[(size_t)k * m + i] = (Vc[(size_t)kk * m + i] * ph).real();
    }
    // Ritz vectors and images: X = Y V, AX = Y W (one streaming pass over
    // the basis per block of kMaxRhs vectors)
    hip_check(hipMemcpyAsync(ydev, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice, c.s), "H2D");
    for (int k0 = 0; k0 < nk; k0 += kMaxRhs) {
      const int kk = std::min(kMaxRhs, nk - k0);
      kc(rows_axpy_multi(c.s, V, m, N, ydev + (int64_t)k0 * m, 1.0, X + (int64_t)k0 * N, N, kk, true), "ritz");
      kc(rows_axpy_multi(c.s, W, m, N, ydev + (int64_t)k0 * m, 1.0, AX + (int64_t)k0 * N, N, kk, true), "ritz");
    }
    phase(1);
    std::vector<double> rn(nk, 0.0);
    std::vector<double*> newv;
    double worst = 0.0;
    // residual norms of the wanted roots (of all Ritz pairs when reporting)
    for (int k = 0; k < (verbose() ? nk : std::min(nk, nroots)); ++k) {
      double* xk = X + (int64_t)k * N;
      double* axk = AX + (int64_t)k * N;
      copy_d(c, Rs, axk, N);
      axpby_(c, Rs, xk, -res.w[k], 1.0, N);
      const double xn = std::sqrt(dotb(xk, xk));
      rn[k] = std::sqrt(std::max(0.0, dotb(Rs, Rs))) / xn;
      if (k < nroots) worst = std::max(worst, rn[k]);
    }
    if (!std::isfinite(worst)) throw Error(-5, "non-finite Davidson residual");
    phase(2);
    if (verbose()) {
      std::fprintf(stderr, "[davidson] it %d m %d", it, m);
      for (int k = 0; k < nk; ++k) std::fprintf(stderr, " w%d=%.12f r=%.2e", k, res.w[k], rn[k]);
      std::fprintf(stderr, "\n");
    }
    if (lowp) {
      if (worst < 0.7 * best_lowp) {
        best_lowp = worst;
        stall = 0;
      } else {
        ++stall;
      }
    }
    if (lowp && (worst < c.opts.tol_eom || stall >= 3 ||
                 (!refreshed && (worst < eig_switch(c) || it >= c.opts.maxit / 2)))) {
      const double wt = refresh(Y, nk);
      refreshed = true;
      best_lowp = 1e300;
      stall = 0;
      if (verbose()) std::fprintf(stderr, "[davidson] it %d fp64 images, true residual %.2e\n", it, wt);
      if (!std::isfinite(wt)) throw Error(-5, "non-finite Davidson residual");
      if (wt < c.opts.tol_eom) {
        res.converged = true;
        break;
      }
      continue;   // Ritz pairs again from the corrected G
    }
    if (!lowp && worst < c.opts.tol_eom) {
      res.converged = true;
      break;
    }
    // restart when the subspace is full: the Ritz vectors and images become
    // the new basis (copied first, orth() works on its arguments in place)
    if (m + nk > maxm) {
      m = 0;
      std::fill(G.begin(), G.end(), 0.0);
      if (!tmpx) {
        tmpx = ar.alloc((int64_t)nb * N);
        tmpa = ar.alloc((int64_t)nb * N);
      }
      copy_d(c, tmpx, X, (int64_t)nk * N);
      copy_d(c, tmpa, AX, (int64_t)nk * N);
      for (int k = 0; k < nk; ++k) orth(tmpx + (int64_t)k * N, tmpa + (int64_t)k * N);
      flush(0, m);
      continue;
    }
    // corrections only for the wanted roots (one block application); the
    // extra Ritz vectors stay in the subspace (and survive restarts) as ballast
    const int m0 = m;
    int r = 0;
    std::vector<double> n0;
    for (int k = 0; k < std::min(nk, nroots); ++k) {
      if (rn[k] < c.opts.tol_eom) continue;
      double* x = Cblk + (int64_t)r * N;
      copy_d(c, x, AX + (int64_t)k * N, N);
      axpby_(c, x, X + (int64_t)k * N, -res.w[k], 1.0, N);
      kc(half_denominator(c.s, x, x, peps, c.o, c.v, res.w[k]), "precondition");
      n0.push_back(std::sqrt(std::max(0.0, dotb(x, x))));
      ++r;
    }
    // block Gram-Schmidt against the (orthonormal) basis; a second pass only
    // when the first removed more than half of some vector's squared norm
    for (int pass = 0; pass < 2 && m0 > 0 && r > 0; ++pass) {
      dots_rows_multi(c, V, m0, Cblk, r, N, false, workm, H);
      sub_rows_multi(c, V, m0, H, Cblk, r, N, hdm);
      bool again = false;
      for (int a = 0; a < r; ++a) {
        double p2 = 0.0;
        for (int k = 0; k < m0; ++k) p2 += H[(size_t)a * m0 + k] * H[(size_t)a * m0 + k];
        if (p2 > 0.5 * n0[a] * n0[a]) again = true;
      }
      if (!again) break;
    }
    for (int a = 0; a < r && m < maxm; ++a) {
      double* x = Cblk + (int64_t)a * N;
      for (int pass = 0; pass < 2 && m > m0; ++pass) {
        dots_rows(c, V + (int64_t)m0 * N, m - m0, x, N, false, work, h);
        sub_rows(c, V + (int64_t)m0 * N, m - m0, h, x, N, hd);
      }
      const double n1 = std::sqrt(std::max(0.0, dotb(x, x)));
      if (!(n0[a] > 0) || n1 < 1e-4 * n0[a] || n1 < 1e-14) continue;
      axpby_(c, V + (int64_t)m * N, x, 1.0 / n1, 0.0, N);
      ++m;
    }
    phase(3);
    flush(m0, m0);
  }
  c.eng->set_lowp(false);
  c.eng->set_bf16(false);
  if (verbose())
    std::fprintf(stderr,
                 "[davidson] %d iterations, %.3f s in operator applications; eig %.3f ritz %.3f residuals %.3f "
                 "corrections %.3f projections %.3f s\n",
                 res.iters, t_apply, t_ph[0], t_ph[1], t_ph[2], t_ph[3], t_ph[4] - t_apply);
  // normalise and hand out the nroots lowest Ritz vectors
  for (int k = 0; k < nroots; ++k) {
    const double xn = std::sqrt(dotb(X + (int64_t)k * N, X + (int64_t)k * N));
    kc(half_unpack(c.s, out[k], X + (int64_t)k * N, c.o, c.v), "unpack");
    axpby_(c, out[k], out[k], 1.0 / xn, 0.0, c.N);
  }
  res.w.resize(nroots);
  (void)nov;
  return res;
}

// Signed value of the largest-magnitude unique parameter (lowest packed index
// on ties) of an amplitude-shaped vector.
__global__ void signed_max_partial(const double* x, int o, int v, int64_t n, double* pv,
                                   int64_t* pi) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int64_t nov = (int64_t)o * v;
  double best = -1.0, bval = 0.0;
  int64_t bidx = INT64_MAX;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t pidx;
    if (e < nov) {
      pidx = e;
    } else {
      int64_t r = e - nov;
      const int b = (int)(r % v); r /= v;
      const int a = (int)(r % v); r /= v;
      const int j = (int)(r % o);
      const int i = (int)(r / o);
      const int64_t P = (int64_t)i * v + a, Q = (int64_t)j * v + b;
      if (P > Q) continue;
      pidx = nov + P * nov - P * (P - 1) / 2 + (Q - P);
    }
    const double a = fabs(x[e]);
    if (a > best || (a == best && pidx < bidx)) { best = a; bval = x[e]; bidx = pidx; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bidx;
  __shared__ double sval[256];
  sval[threadIdx.x] = bval;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const int o2 = threadIdx.x + s;
      if (sv[o2] > sv[threadIdx.x] || (sv[o2] == sv[threadIdx.x] && si[o2] < si[threadIdx.x])) {
        sv[threadIdx.x] = sv[o2];
        si[threadIdx.x] = si[o2];
        sval[threadIdx.x] = sval[o2];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[2 * blockIdx.x] = sv[0];
    pv[2 * blockIdx.x + 1] = sval[0];
    pi[blockIdx.x] = si[0];
  }
}

// ------------------------------------------------ learned doubles guess
// Features of doubles index e = ((i o + j) v + a) v + b: e_i, e_j, e_a, e_b,
// D, (ia|jb), (ib|ja), -(ia|jb)/D, standardised with mu and 1/sd; g is the
// bare block (ia|jb) stored [i][a][j][b].
__global__ void t2_features_kernel(const double* __restrict__ g, const double* __restrict__ eps,
                                   int o, int v, const float* __restrict__ mu,
                                   const float* __restrict__ isd, float* __restrict__ F) {
  const int64_t tot = (int64_t)o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const double ei = eps[i], ej = eps[j], ea = eps[o + a], eb = eps[o + b];
    const double D = ea + eb - ei - ej;
    const double giajb = g[(((int64_t)i * v + a) * o + j) * v + b];
    const double gibja = g[(((int64_t)i * v + b) * o + j) * v + a];
    const double f[8] = {ei, ej, ea, eb, D, giajb, gibja, -giajb / D};
#pragma unroll
    for (int k = 0; k < 8; ++k) F[e * 8 + k] = (float)((f[k] - (double)mu[k]) * (double)isd[k]);
  }
}

// z = (-D t - (ia|jb)) / scale (target) or t = -((ia|jb) + scale z) / D (guess);
// g: (ia|jb) stored [i][a][j][b]
__global__ void t2_map_kernel(const double* __restrict__ g, const double* __restrict__ eps, int o,
                              int v, double* __restrict__ t2, float* __restrict__ z, double scale,
                              int to_amplitudes) {
  const int64_t tot = (int64_t)o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    const int b = (int)(r % v); r /= v;
    const int a = (int)(r % v); r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    const double D = eps[o + a] + eps[o + b] - eps[i] - eps[j];
    const double giajb = g[(((int64_t)i * v + a) * o + j) * v + b];
    if (to_amplitudes)
      t2[e] = -(giajb + scale * (double)z[e]) / D;
    else
      z[e] = (float)((-D * t2[e] - giajb) / scale);
  }
}

static float* feature_norm(Ctx& c, const float* mu, const float* sd) {
  float h[16];
  for (int k = 0; k < 8; ++k) {
    h[k] = mu ? mu[k] : 0.0f;
    const float s = sd ? sd[k] : 1.0f;
    if (!(s > 0.0f)) throw Error(-1, "feature scales must be positive");
    h[8 + k] = 1.0f / s;
  }
  float* d = (float*)c.eng->arena().alloc(8);
  hip_check(hipMemcpyAsync(d, h, sizeof(h), hipMemcpyHostToDevice, c.s), "H2D");
  sync(c);
  return d;
}

static double signed_max(Ctx& c, const double* x) {
  const int nbk = 256;
  ArenaScope sc(c.eng->arena());
  double* pv = c.eng->arena().alloc(2 * nbk);
  int64_t* pi = (int64_t*)c.eng->arena().alloc(nbk);
  hipLaunchKernelGGL(signed_max_partial, dim3(nbk), dim3(256), 0, c.s, x, c.o, c.v, c.N, pv, pi);
  hip_check(hipGetLastError(), "signed_max");
  std::vector<double> hv(2 * nbk);
  std::vector<int64_t> hi(nbk);
  hip_check(hipMemcpyAsync(hv.data(), pv, 2 * nbk * sizeof(double), hipMemcpyDeviceToHost, c.s), "D2H");
  hip_check(hipMemcpyAsync(hi.data(), pi, nbk * sizeof(int64_t), hipMemcpyDeviceToHost, c.s), "D2H");
  sync(c);
  double best = -1.0, val = 0.0;
  int64_t bi = INT64_MAX;
  for (int k = 0; k < nbk; ++k)
    if (hv[2 * k] > best || (hv[2 * k] == best && hi[k] < bi)) {
      best = hv[2 * k];
      val = hv[2 * k + 1];
      bi = hi[k];
    }
  return val;
}

static int eom(Ctx& c, int side, int nroots, double* omega, int* iters) {
  if (nroots != c.nroots) {
    c.R.clear();
    c.L.clear();
    c.have_right = c.have_left = c.gauged = false;
    // pairs that involve excited states are stale; the ground-state gradient
    // (pair (0, 0)) depends on the amplitudes only
    for (auto it = c.pairs.begin(); it != c.pairs.end();) {
      if (it->first.first != 0 || it->first.second != 0) it = c.pairs.erase(it); else ++it;
    }
    for (int k = 0; k < nroots; ++k) {
      c.R.push_back(palloc(c, c.N));
      c.L.push_back(palloc(c, c.N));
    }
    c.nroots = nroots;
  }
  int status = CC_OK, itsum = 0;
  Tape tp(c);
  auto guesses = [&](std::map<int, double*>& gm) {
    std::vector<double*> gv;
    for (auto& kv : gm)
      if (kv.first >= 1 && kv.first <= nroots) gv.push_back(kv.second);
    return gv;
  };
  if (side & CC_RIGHT) {
    std::vector<double*> gr = guesses(c.guess_R);
    Ritz r = davidson(c, nroots, [&](const double* x, double* y, int k) { tp.right_block(x, y, k); }, c.R,
                      gr.empty() ? nullptr : &gr, tp.deps);
    c.guess_R.clear();
    if (r.complex_root) return CC_ERR_COMPLEX_ROOT;
    c.omega_r = r.w;
    c.have_right = true;
    c.gauged = false;
    itsum += r.iters;
    if (!r.converged) status = CC_NOT_CONVERGED;
  }
  if (side & CC_LEFT) {
    std::vector<double*> gl = guesses(c.guess_L);
    if (gl.empty() && c.have_right) gl = c.R;
    Ritz r = davidson(c, nroots, [&](const double* x, double* y, int k) { tp.left_block(x, y, k); },
                      c.L, gl.empty() ? nullptr : &gl, tp.deps);
    c.guess_L.clear();
    if (r.complex_root) return CC_ERR_COMPLEX_ROOT;
    c.omega_l = r.w;
    c.have_left = true;
    c.gauged = false;
    itsum += r.iters;
    if (!r.converged) status = CC_NOT_CONVERGED;
  }
  if (iters) *iters = itsum;
  if (c.have_right && c.have_left && !c.gauged) {
    // gauge of R: unit norm (already), largest parameter positive
    for (int k = 0; k < nroots; ++k) {
      const double sv = signed_max(c, c.R[k]);
      if (sv < 0) axpby_(c, c.R[k], c.R[k], -1.0, 0.0, c.N);
    }
    // biorthonormalise L: L <- S^{-1} L with S_kl = L_k . R_l
    std::vector<double> S((size_t)nroots * nroots), Id((size_t)nroots * nroots, 0.0);
    for (int k = 0; k < nroots; ++k)
      for (int l = 0; l < nroots; ++l) S[(size_t)k * nroots + l] = dot_bio(c, c.L[k], c.R[l]);
    for (int k = 0; k < nroots; ++k) Id[(size_t)k * nroots + k] = 1.0;
    if (!lu_solve(S, Id, nroots, nroots)) throw Error(-5, "left and right states not biorthogonalisable");
    {
      ArenaScope sc(c.eng->arena());
      double* tmp = c.eng->arena().alloc((int64_t)nroots * c.N);
      for (int k = 0; k < nroots; ++k) {
        kc(fill(c.s, tmp + (int64_t)k * c.N, 0.0, c.N), "fill");
        for (int l = 0; l < nroots; ++l)
          axpby_(c, tmp + (int64_t)k * c.N, c.L[l], Id[(size_t)k * nroots + l], 1.0, c.N);
      }
      for (int k = 0; k < nroots; ++k) copy_d(c, c.L[k], tmp + (int64_t)k * c.N, c.N);
    }
    c.R0.assign(nroots, 0.0);
    for (int k = 0; k < nroots; ++k) c.R0[k] = energy_jvp(c, c.t, c.R[k]) / c.omega_r[k];
    c.gauged = true;
  }
  if (omega) {
    const std::vector<double>& w = (side & CC_RIGHT) ? c.omega_r : c.omega_l;
    for (int k = 0; k < nroots; ++k) omega[k] = w[k];
  }
  return status;
}

// --------------------------------------------------------- linear solver
// Solves T(x_r) = b_r for k right-hand sides (T on amplitude-shaped vectors,
// biorthonormal metric, or on plain vectors of length n) by a Galerkin
// projection on one growing subspace V shared by all of them, with images
// W = T(V): for each r, G y_r = V^T b_r with G = V^T W, x_r = V y_r.  Each
// iteration extends V by the preconditioned residuals of the systems not yet
// converged and images them in one block application of T, so that k systems
// share every pass through the operator.  A system's solution is frozen once
// its residual meets the tolerance.  When the subspace is full it restarts
// from the current solutions.
//
// mixed: the images come from the low-precision operator.  When a residual
// computed from them reaches its rounding floor (eig_switch relative, or a
// stall), and whenever it meets the tolerance, the current solutions
// X = Y V get fp64 images and their true residuals are measured; the basis
// images then get the rank-k correction W <- W + Z^T D with D = T64(X) - Y W
// and Z = (Y Y^T)^-1 Y (Z Y^T = I), so that the images of the solutions become
// exact (G gets the same update) and the subspace is kept.  Only a true
// residual below the tolerance ends a system's solve.
constexpr int kMaxBlockRhs = 8;
static int linsolve_core(Ctx& c, int64_t n, bool packed, int k,
                         const std::function<void(const double*, double*, int)>& T,
                         const std::function<void(double*, const double*)>& precond,
                         const double* B, double* X, double tol, int maxit, int* iters,
                         bool mixed_images) {
  if (k < 1 || k > kMaxBlockRhs) throw Error(-1, "linear solver block size out of range");
  Arena& ar = c.eng->arena();
  ArenaScope sc(ar);
  // subspace size: as the Davidson solver's (davidson_max), at least room
  // for four blocks of k vectors
  const int maxm = std::min({kMaxRows - kMaxBlockRhs, 120, std::max(c.opts.davidson_max, 4 * k + 4)});
  double* V = ar.alloc((int64_t)maxm * n);
  double* W = ar.alloc((int64_t)maxm * n);
  double* Rr = ar.alloc((int64_t)k * n);      // residuals T x_r - b_r
  double* Cb = ar.alloc((int64_t)k * n);      // new basis vectors / fp64 images
  double* workm = ar.alloc((int64_t)k * n + (int64_t)k * maxm);
  double* Db = ar.alloc((int64_t)k * n + (int64_t)k * maxm);   // second work block
  double* hdm = ar.alloc((int64_t)k * maxm);
  double* ydev = ar.alloc((int64_t)k * maxm);
  double* zdev = ar.alloc((int64_t)k * maxm);
  auto dotf = [&](const double* p, const double* q) {
    return packed ? dot_bio(c, p, q) : dot_plain(c, p, q, n);
  };
  std::vector<double> G((size_t)maxm * maxm, 0.0), H, bvm((size_t)k * maxm, 0.0);
  std::vector<double> bn(k), goal(k), best(k, 1e300), rn(k, 0.0);
  std::vector<int> stall(k, 0), conv(k, 0), it_of(k, 0);
  std::vector<char> refreshed(k, 0);
  int m = 0;
  c.eng->set_lowp(mixed_images);
  c.eng->set_bf16(mixed_images && solver_bf16(c));
  for (int r = 0; r < k; ++r) {
    const double* b = B + (int64_t)r * n;
    bn[r] = std::sqrt(std::max(dotf(b, b), 0.0));
    goal[r] = tol * std::max(1.0, bn[r]);
    kc(fill(c.s, X + (int64_t)r * n, 0.0, n), "fill");
    axpby_(c, Rr + (int64_t)r * n, b, -1.0, 0.0, n);   // residual of x = 0
    if (bn[r] < goal[r]) conv[r] = 1;                  // x = 0 is exact
  }
  // images of rows [m0, m), then the new rows and columns of G and V^T b
  auto extend = [&](int m0) {
    const int r = m - m0;
    if (r <= 0) return;
    T(V + (int64_t)m0 * n, W + (int64_t)m0 * n, r);
    dots_rows_multi(c, V, m, W + (int64_t)m0 * n, r, n, packed, workm, H);
    for (int jj = 0; jj < r; ++jj)
      for (int a = 0; a < m; ++a) G[(size_t)a * maxm + m0 + jj] = H[(size_t)jj * m + a];
    dots_rows_multi(c, W, m, V + (int64_t)m0 * n, r, n, packed, workm, H);
    for (int jj = 0; jj < r; ++jj)
      for (int a = 0; a < m; ++a) G[(size_t)(m0 + jj) * maxm + a] = H[(size_t)jj * m + a];
    dots_rows_multi(c, V + (int64_t)m0 * n, r, B, k, n, packed, workm, H);
    for (int q = 0; q < k; ++q)
      for (int jj = 0; jj < r; ++jj) bvm[(size_t)q * maxm + m0 + jj] = H[(size_t)q * r + jj];
  };
  // appends the nv vectors of Cb to the basis (block Gram-Schmidt against V,
  // then one by one among themselves); returns how many were kept
  auto append = [&](int nv) {
    if (packed)
      for (int a = 0; a < nv; ++a)
        kc(apply_metric(c.s, Cb + (int64_t)a * n, Cb + (int64_t)a * n, c.o, c.v, 2), "symmetrise");
    std::vector<double> n0(nv);
    for (int a = 0; a < nv; ++a) n0[a] = std::sqrt(std::max(0.0, dotf(Cb + (int64_t)a * n, Cb + (int64_t)a * n)));
    const int m0 = m;
    for (int pass = 0; pass < 2 && m0 > 0; ++pass) {
      dots_rows_multi(c, V, m0, Cb, nv, n, packed, workm, H);
      sub_rows_multi(c, V, m0, H, Cb, nv, n, hdm);
      bool again = false;
      for (int a = 0; a < nv; ++a) {
        double p2 = 0.0;
        for (int q = 0; q < m0; ++q) p2 += H[(size_t)a * m0 + q] * H[(size_t)a * m0 + q];
        if (p2 > 0.5 * n0[a] * n0[a]) again = true;
      }
      if (!again) break;
    }
    std::vector<double> h;
    for (int a = 0; a < nv && m < maxm; ++a) {
      double* x = Cb + (int64_t)a * n;
      for (int pass = 0; pass < 2 && m > m0; ++pass) {
        dots_rows(c, V + (int64_t)m0 * n, m - m0, x, n, packed, workm, h);
        sub_rows(c, V + (int64_t)m0 * n, m - m0, h, x, n, hdm);
      }
      const double n1 = std::sqrt(std::max(0.0, dotf(x, x)));
      if (!(n0[a] > 0) || n1 < 1e-12 * n0[a] || n1 < 1e-300) continue;
      axpby_(c, V + (int64_t)m * n, x, 1.0 / n1, 0.0, n);
      ++m;
    }
    return m - m0;
  };
  int status = CC_NOT_CONVERGED;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    std::vector<int> act;
    for (int r = 0; r < k; ++r)
      if (!conv[r]) act.push_back(r);
    if (act.empty()) { status = CC_OK; break; }
    const int na = (int)act.size();
    // restart from the current solutions when the new vectors do not fit
    if (m + na > maxm) {
      m = 0;
      std::fill(G.begin(), G.end(), 0.0);
      for (int a = 0; a < na; ++a) copy_d(c, Cb + (int64_t)a * n, X + (int64_t)act[a] * n, n);
      const int kept = append(na);
      extend(0);
      (void)kept;
    }
    // next basis vectors: preconditioned residuals of the open systems
    for (int a = 0; a < na; ++a) precond(Cb + (int64_t)a * n, Rr + (int64_t)act[a] * n);
    const int m0 = m;
    if (append(na) == 0) break;   // no new direction: stagnated
    extend(m0);
    for (int pass = 0;; ++pass) {
      // Galerkin solutions of the open systems
      std::vector<double> Gm((size_t)m * m), Y((size_t)m * na);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) Gm[(size_t)a * m + b] = G[(size_t)a * maxm + b];
      for (int q = 0; q < na; ++q)
        for (int a = 0; a < m; ++a) Y[(size_t)a * na + q] = bvm[(size_t)act[q] * maxm + a];
      if (!lu_solve(Gm, Y, m, na)) throw Error(-5, "singular projected linear system");
      std::vector<double> Yr((size_t)na * m);   // row q = coefficients of system act[q]
      for (int q = 0; q < na; ++q)
        for (int a = 0; a < m; ++a) Yr[(size_t)q * m + a] = Y[(size_t)a * na + q];
      hip_check(hipMemcpyAsync(ydev, Yr.data(), Yr.size() * sizeof(double), hipMemcpyHostToDevice, c.s),
                "H2D");
      double worst = 0.0;
      for (int q = 0; q < na; ++q) {
        const int r = act[q];
        kc(rows_axpy_multi(c.s, V, m, n, ydev + (int64_t)q * m, 1.0, X + (int64_t)r * n, n, 1, true), "combine");
        kc(rows_axpy_multi(c.s, W, m, n, ydev + (int64_t)q * m, 1.0, Rr + (int64_t)r * n, n, 1, true), "combine");
        axpby_(c, Rr + (int64_t)r * n, B + (int64_t)r * n, -1.0, 1.0, n);
        rn[r] = std::sqrt(std::max(0.0, dotf(Rr + (int64_t)r * n, Rr + (int64_t)r * n)));
        if (!std::isfinite(rn[r])) throw Error(-5, "non-finite linear-solver residual");
        worst = std::max(worst, rn[r] / goal[r]);
      }
      if (verbose()) {
        std::fprintf(stderr, "[linsolve] it %d m %d", it, m);
        for (int q = 0; q < na; ++q) std::fprintf(stderr, " |r%d| %.3e", act[q], rn[act[q]]);
        std::fprintf(stderr, "\n");
      }
      if (!mixed_images) {
        for (int q = 0; q < na; ++q)
          if (rn[act[q]] < goal[act[q]]) { conv[act[q]] = 1; it_of[act[q]] = it; }
        break;
      }
      // mixed: residuals from the low-precision images never end a solve by
      // themselves; they decide when the solutions get fp64 images
      bool want = false;
      for (int q = 0; q < na; ++q) {
        const int r = act[q];
        if (rn[r] < 0.7 * best[r]) { best[r] = rn[r]; stall[r] = 0; } else { ++stall[r]; }
        if (rn[r] < goal[r] || stall[r] >= 3 || (!refreshed[r] && rn[r] < eig_switch(c) * bn[r]))
          want = true;
      }
      if (!want) break;
      // fp64 images of the open solutions, true residuals, rank-na correction
      for (int q = 0; q < na; ++q) copy_d(c, workm + (int64_t)q * n, X + (int64_t)act[q] * n, n);
      c.eng->set_lowp(false);
      T(workm, Cb, na);
      c.eng->set_lowp(true);
      std::vector<double> rt(na);
      for (int q = 0; q < na; ++q) {
        const int r = act[q];
        double* d = Cb + (int64_t)q * n;
        refreshed[r] = 1;
        best[r] = 1e300;
        stall[r] = 0;
        axpby_(c, d, B + (int64_t)r * n, -1.0, 1.0, n);            // true residual
        rt[q] = std::sqrt(std::max(0.0, dotf(d, d)));
        if (!std::isfinite(rt[q])) throw Error(-5, "non-finite linear-solver residual");
        axpby_(c, d, Rr + (int64_t)r * n, -1.0, 1.0, n);           // D = true - computed
        if (verbose()) std::fprintf(stderr, "[linsolve] it %d fp64 image of %d, true |r| %.3e\n", it, r, rt[q]);
      }
      // Z = (Y Y^T)^-1 Y over the open systems (solutions x = 0 have exact
      // images already and are left out)
      std::vector<int> nz;
      for (int q = 0; q < na; ++q) {
        double yy = 0.0;
        for (int a = 0; a < m; ++a) yy += Yr[(size_t)q * m + a] * Yr[(size_t)q * m + a];
        if (yy > 0.0) nz.push_back(q);
      }
      if (!nz.empty()) {
        const int kz = (int)nz.size();
        std::vector<double> S((size_t)kz * kz, 0.0), Z((size_t)kz * m);
        for (int a = 0; a < kz; ++a)
          for (int b = 0; b < kz; ++b)
            for (int i = 0; i < m; ++i)
              S[(size_t)a * kz + b] += Yr[(size_t)nz[a] * m + i] * Yr[(size_t)nz[b] * m + i];
        for (int a = 0; a < kz; ++a)
          for (int i = 0; i < m; ++i) Z[(size_t)a * m + i] = Yr[(size_t)nz[a] * m + i];
        if (!lu_solve(S, Z, kz, m)) throw Error(-5, "dependent linear-solver solutions");
        // D rows of the systems in nz, contiguous
        const double* Dz = Cb;
        if (kz != na) {
          for (int a = 0; a < kz; ++a) copy_d(c, workm + (int64_t)a * n, Cb + (int64_t)nz[a] * n, n);
          Dz = workm;
        }
        hip_check(hipMemcpyAsync(zdev, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice, c.s),
                  "H2D");
        kc(gemm_f64(c.s, true, false, m, (int)n, kz, 1, 1.0, zdev, m, 0, Dz, n, 0, 1.0, W, n, 0),
           "image update");
        dots_rows_multi(c, V, m, Dz, kz, n, packed, Db, H);
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) {
            double acc = 0.0;
            for (int q = 0; q < kz; ++q) acc += H[(size_t)q * m + a] * Z[(size_t)q * m + b];
            G[(size_t)a * maxm + b] += acc;
          }
      }
      bool all = true;
      for (int q = 0; q < na; ++q) {
        const int r = act[q];
        if (rt[q] < goal[r]) {
          axpby_(c, Rr + (int64_t)r * n, Cb + (int64_t)q * n, 1.0, 1.0, n);   // true residual
          conv[r] = 1;
          it_of[r] = it;
        } else {
          all = false;
        }
      }
      if (all) break;
      if (pass >= 2) {
        // after three corrected solves in a row the next basis vectors come
        // from the true residuals
        for (int q = 0; q < na; ++q)
          if (!conv[act[q]]) axpby_(c, Rr + (int64_t)act[q] * n, Cb + (int64_t)q * n, 1.0, 1.0, n);
        break;
      }
      // solve again with the corrected images: the converged systems drop out
      std::vector<int> still;
      for (int q = 0; q < na; ++q)
        if (!conv[act[q]]) still.push_back(act[q]);
      // (the remaining pass works on the systems still open)
      if (still.size() != act.size()) break;
    }
  }
  bool all = true;
  for (int r = 0; r < k; ++r) {
    if (!conv[r]) all = false;
    if (iters) iters[r] = conv[r] ? std::max(it_of[r], 1) : std::min(it, maxit);
  }
  if (all) status = CC_OK;
  c.eng->set_lowp(false);
  c.eng->set_bf16(false);
  return status;
}

// T X = B for k right-hand sides.  Amplitude-shaped systems (packed) run in
// the half layout (singles and doubles (ia) <= (jb), where the biorthonormal
// product is the plain dot product), so every pass over the subspace moves
// half the bytes; vectors are unpacked to the full symmetric layout for T and
// the preconditioner.
static int linsolve_block(Ctx& c, int64_t n, bool packed, int k,
                          const std::function<void(const double*, double*, int)>& T,
                          const std::function<void(double*, const double*)>& precond,
                          const double* B, double* X, double tol, int maxit, int* iters,
                          bool mixed_images) {
  if (!packed) return linsolve_core(c, n, false, k, T, precond, B, X, tol, maxit, iters, mixed_images);
  if (k < 1 || k > kMaxBlockRhs) throw Error(-1, "linear solver block size out of range");
  const int64_t nh = half_len(c);
  Arena& ar = c.eng->arena();
  ArenaScope sc(ar);
  double* Fin = ar.alloc((int64_t)k * n);
  double* Fout = ar.alloc((int64_t)k * n);
  double* Bh = ar.alloc((int64_t)k * nh);
  double* Xh = ar.alloc((int64_t)k * nh);
  for (int r = 0; r < k; ++r) {
    copy_d(c, Fin, B + (int64_t)r * n, n);
    kc(apply_metric(c.s, Fin, Fin, c.o, c.v, 2), "symmetrise");
    kc(half_pack(c.s, Bh + (int64_t)r * nh, Fin, c.o, c.v), "pack");
  }
  const int kt = transform_batch(c);
  auto Th = [&](const double* xh, double* yh, int r) {
    for (int z0 = 0; z0 < r; z0 += kt) {
      const int rr = std::min(kt, r - z0);
      for (int z = 0; z < rr; ++z)
        kc(half_unpack(c.s, Fin + (int64_t)z * n, xh + (int64_t)(z0 + z) * nh, c.o, c.v), "unpack");
      T(Fin, Fout, rr);
      for (int z = 0; z < rr; ++z)
        kc(half_pack(c.s, yh + (int64_t)(z0 + z) * nh, Fout + (int64_t)z * n, c.o, c.v), "pack");
    }
  };
  auto preh = [&](double* yh, const double* xh) {
    kc(half_unpack(c.s, Fin, xh, c.o, c.v), "unpack");
    precond(Fout, Fin);
    kc(half_pack(c.s, yh, Fout, c.o, c.v), "pack");
  };
  const int st = linsolve_core(c, nh, false, k, Th, preh, Bh, Xh, tol, maxit, iters, mixed_images);
  for (int r = 0; r < k; ++r) kc(half_unpack(c.s, X + (int64_t)r * n, Xh + (int64_t)r * nh, c.o, c.v), "unpack");
  return st;
}

// Single right-hand side.
static int linsolve(Ctx& c, int64_t n, bool packed, const std::function<void(const double*, double*)>& T,
                    const std::function<void(double*, const double*)>& precond, const double* b,
                    double* x, double tol, int maxit, int* iters, bool mixed_images = false) {
  auto Tb = [&](const double* X, double* Y, int kk) {
    for (int z = 0; z < kk; ++z) T(X + (int64_t)z * n, Y + (int64_t)z * n);
  };
  return linsolve_block(c, n, packed, 1, Tb, precond, b, x, tol, maxit, iters, mixed_images);
}

// T(x) = b in the context's precision: plain fp64 linsolve, or with
// low-precision images and fp64 image corrections (mixed precision).
static int linsolve_refined(Ctx& c, int64_t n, bool packed,
                            const std::function<void(const double*, double*)>& T,
                            const std::function<void(double*, const double*)>& precond,
                            const double* b, double* x, double tol, int maxit, int* iters) {
  return linsolve(c, n, packed, T, precond, b, x, tol, maxit, iters, mixed(c));
}

// ------------------------------------------------------ orbital rotation
// The Hamiltonian exp(kappa) H exp(-kappa) to first order in kappa (exact
// for derivatives at kappa = 0), K_ai = kappa_ai, K_ia = -kappa_ai: the factor
// changes by db[P] = K B[P] + B[P] K^T, the one-electron integrals
// h = f - 2 J[B] + X[B] (implied by the canonical Fock matrix f) by
// K h + h K^T, and the Fock matrix of the rotated Hamiltonian, built over the
// same occupied range, is
//   fr = f + K h + h K^T + 2 (J(db, B) + J(B, db)) - (X(db, B) + X(B, db))
// with J(Y, Z)_pq = sum_P (sum_k Y[P][k][k]) Z[P][p][q] and
// X(Y, Z)_pq = sum_P sum_k Y[P][p][k] Z[P][k][q].  Derivatives of a function
// of (f, B) along kappa are reverse sweeps of this graph seeded on fr and db.
struct RotNodes { int kap, fr, db; };
static RotNodes rotation_graph(Graph& G, Ctx& c, const Tensor& kappa) {
  const int64_t o = c.o, v = c.v, n = c.n, P = c.naux;
  const Range O{0, o}, V{o, v}, A{0, n}, AP{0, P};
  RotNodes r;
  r.kap = G.leaf(kappa);
  const int fl = G.leaf(c.f), bl = G.leaf(c.B);
  const int trb = G.node({P}, {lin(1, op(bl, "Pkk", {AP, O, O}), "P")});
  const int h = G.node({n, n}, {lin(1, op(fl, "pq"), "pq"),
                                mul(-2, op(trb, "P"), op(bl, "Ppq"), "pq"),
                                mul(1, op(bl, "Ppk", {AP, A, O}), op(bl, "Pkq", {AP, O, A}), "pq")});
  const int K = G.node({n, n}, {lin(1, op(r.kap, "ia"), "ai", {V, O}), lin(-1, op(r.kap, "ia"), "ia", {O, V})});
  r.db = G.node({P, n, n}, {mul(1, op(K, "pt"), op(bl, "Ptq"), "Ppq"),
                            mul(1, op(bl, "Ppt"), op(K, "qt"), "Ppq")});
  const int trdb = G.node({P}, {lin(1, op(r.db, "Pkk", {AP, O, O}), "P")});
  r.fr = G.node({n, n}, {lin(1, op(fl, "pq"), "pq"), mul(1, op(K, "pt"), op(h, "tq"), "pq"),
                         mul(1, op(h, "pt"), op(K, "qt"), "pq"),
                         mul(2, op(trdb, "P"), op(bl, "Ppq"), "pq"),
                         mul(2, op(trb, "P"), op(r.db, "Ppq"), "pq"),
                         mul(-1, op(r.db, "Ppk", {AP, A, O}), op(bl, "Pkq", {AP, O, A}), "pq"),
                         mul(-1, op(bl, "Ppk", {AP, A, O}), op(r.db, "Pkq", {AP, O, A}), "pq")});
  return r;
}

// ------------------------------------------------------------- multipliers
static PairData& pair_of(Ctx& c, int i, int j) {
  PairData& p = c.pairs[{i, j}];
  if (!p.zeta) {
    p.zeta = palloc(c, c.N);
    p.gamma = palloc(c, c.N);
    p.eta_t = palloc(c, c.N);
    p.kbar = palloc(c, (int64_t)c.o * c.v);
    p.eta_k = palloc(c, (int64_t)c.o * c.v);
    p.dtrans = palloc(c, (int64_t)c.n * c.n);
    p.Fbar = palloc(c, (int64_t)c.n * c.n);
    p.Deff = palloc(c, (int64_t)c.n * c.n);
  }
  return p;
}


// M[i][i] += a for the occupied i (e.g. the derivative of the Hartree-Fock
// energy E_HF = 2 sum_i f_ii - sum_ij (2 g_iijj - g_ijji) by the Fock leaf)
__global__ void diag_occ_add_kernel(double* M, int64_t n, int o, double a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= o) return;
  M[i * n + i] += a;
}

// The vvvv block d Phi / d W[c][d][a][b] from its factors, as a node of G:
// the ladder sum_cd t_ij^cd W[c][d][a][b] is the only place W enters the
// residual, so its adjoint is t2 (and R2 along R_jr) times the ladder
// output's adjoint.
// Only the rows c in [c0, c0 + cc) of its first index are formed (cc = v
// for the whole block).
static int vvvv_density(Graph& G, Ctx& c, const PairData& P, int64_t c0 = 0, int64_t cc = -1) {
  const int64_t o = c.o, v = c.v, o2v2 = o * o * v * v;
  if (cc < 0) cc = v;
  const Range O{0, o}, V{0, v}, Cc{c0, cc};
  const int t2 = G.leaf(T2of(c, c.t));
  const int y0 = G.leaf(tview(P.ylad, {o, o, v, v}));
  std::vector<Term> terms{mul(1, op(t2, "ijcd", {O, O, Cc, V}), op(y0, "ijab"), "cdab")};
  if (P.nlad > 1) {
    const int r2 = G.leaf(T2of(c, c.R[P.jr]));
    const int y1 = G.leaf(tview(P.ylad + o2v2, {o, o, v, v}));
    terms.push_back(mul(1, op(r2, "ijcd", {O, O, Cc, V}), op(y1, "ijab"), "cdab"));
  }
  return G.node({cc, v, v, v}, terms);
}

// rows of the vvvv block formed at a time: about 4 GB of them
static int64_t vvvv_chunk(const Ctx& c) {
  const double row = (double)c.v * c.v * c.v * 8.0;
  return std::max<int64_t>(1, std::min<int64_t>(c.v, (int64_t)(4e9 / row)));
}

// d Phi / d B[P] from the bare blocks W[c][d][a][b] = sum_P B_ac B_bd,
// Wov[c][d][k][b] = sum_P B_kc B_bd, Gov[k][c][l][d] = sum_P B_kc B_ld (each
// product rule term), and, for the energy Lagrangian, from E_HF's
// two-electron part -sum_P [2 (sum_i B_ii)^2 - sum_ij B_ij B_ji]; added to
// the adjoint the factor leaves already hold.
static void fold_bare_adjoints(Ctx& c, PairData& P) {
  const int64_t o = c.o, v = c.v, n = c.n, Pn = c.naux;
  const Range AP{0, Pn}, O{0, o}, V{o, v};
  ArenaScope sc(c.eng->arena());
  Graph G(*c.eng);
  const int b = G.leaf(c.B);
  const int bb = G.leaf(tview(P.Bbar, {Pn, n, n}));
  const int gwov = G.leaf(tview(P.gWov, {v, v, o, v}));
  const int ggov = G.leaf(tview(P.gGov, {o, v, o, v}));
  Engine& e = *c.eng;
  // vvvv, formed a block of rows c at a time
  const int64_t cch = vvvv_chunk(c);
  for (int64_t c0 = 0; c0 < v; c0 += cch) {
    const int64_t cc = std::min(cch, v - c0);
    ArenaScope s2(c.eng->arena());
    const int n0 = G.size();
    const int gw = vvvv_density(G, c, P, c0, cc);
    const Range Vc{o + c0, cc};
    e.contract(1.0, G.view(op(gw, "cdab")), G.view(op(b, "Pbd", {AP, V, V})),
               G.view(op(bb, "Pac", {AP, V, Vc})));
    e.contract(1.0, G.view(op(gw, "cdab")), G.view(op(b, "Pac", {AP, V, Vc})),
               G.view(op(bb, "Pbd", {AP, V, V})));
    G.truncate(n0);
  }
  e.contract(1.0, G.view(op(gwov, "cdkb")), G.view(op(b, "Pbd", {AP, V, V})), G.view(op(bb, "Pkc", {AP, O, V})));
  e.contract(1.0, G.view(op(gwov, "cdkb")), G.view(op(b, "Pkc", {AP, O, V})), G.view(op(bb, "Pbd", {AP, V, V})));
  e.contract(1.0, G.view(op(ggov, "kcld")), G.view(op(b, "Pld", {AP, O, V})), G.view(op(bb, "Pkc", {AP, O, V})));
  e.contract(1.0, G.view(op(ggov, "kcld")), G.view(op(b, "Pkc", {AP, O, V})), G.view(op(bb, "Pld", {AP, O, V})));
  if (P.hf_term) {
    // d/dB[P][p][q] = -4 s[P] delta_pq + 2 B[P][q][p]  (p, q occupied)
    const int s = G.node({Pn}, {lin(1, op(b, "Pkk", {AP, O, O}), "P")});
    e.linear(-4.0, G.view(op(s, "P")), G.view(op(bb, "Pkk", {AP, O, O})));
    e.linear(2.0, G.view(op(b, "Pji", {AP, O, O})), G.view(op(bb, "Pij", {AP, O, O})));
  }
}

// Multipliers of one Lagrangian per pair (i1, j1):
//  * i1 != j1 >= 1: coupling F_ij, Phi = zeta.Omega + gamma.(A R_j), overlap
//    of <L_i| with the right state j (Sec. II B);
//  * j1 = 0 < i1: coupling F_i0 with the CC ground state exp(T)|HF> (R0 = 1,
//    R = 0, no EOM condition, gamma = 0); A^T zeta = -L_i has the closed-form
//    solution zeta = -L_i / omega_i (L_i is a left eigenvector) (Sec. II C);
//  * i1 = j1: gradient of the state energy E_j = E0 + L_j.(A R_j) (E0 alone
//    for j1 = 0): Phi = E0 + zeta.Omega + L_j.(A R_j), no overlap term, so
//    eta_t = dE0/dt + F(L_j) R_j and eta_kappa = d Phi / d kappa;
//  * i1 = 0 < j1: coupling F_0j of the ground-state left state
//    <HF| (1 + Lambda) exp(-T), the left eigenvector (1, Lambda) of the
//    Jacobian bordered by the reference row (eq. nac with i = 0), Lambda from
//    A^T Lambda = -eta (solved first, kept in the context).  Its reference
//    weight brings R0_j into the overlap, so the excited-state condition keeps
//    its reference row eta.R_j - omega_j R0_j, with multiplier 1/omega_j:
//    Phi gains eta(t; f, g).R_j / omega_j (the energy's derivative along
//    R_j), gamma = Lambda/omega_j, and the transition density gains the
//    reference row R0_j dE/df + d(eta.R_j)/df (its first term cancels the
//    E(f) (Lambda . R_j) = -R0_j E(f) of the Lambda part).
// All pairs share one recording of the residual graph and one forward
// derivative along each right state R_j they use; their zeta equations
// A^T zeta = -eta_t (eq. amplituderelax) are solved together, in blocks of up
// to kMaxBlockRhs right-hand sides that go through each left transform as one
// batch.  iters: [npairs][2] (zeta, kappa-bar iterations).
// The energy graph at the current amplitudes with its forward derivative
// along the right state j: te is dE/dt . R_j = eta(t; f, g) . R_j.
struct EnergyTangent {
  Graph G;
  EnergyNodes en;
  int te = -1;
  EnergyTangent(Ctx& c, int j) : G(*c.eng) {
    en = energy_graph(G, c, T1of(c, c.t), T2of(c, c.t));
    const int r1 = G.leaf(T1of(c, c.R[j])), r2 = G.leaf(T2of(c, c.R[j]));
    te = G.jvp({{en.t1, r1}, {en.t2, r2}}).at(en.e);
  }
};

struct PairJob {
  int i1, j1;
  bool grad_mode, has_right;
  bool ground_bra = false;   // i1 = 0 < j1: the bra <HF| (1 + Lambda) exp(-T)
  const double* Lleft = nullptr;   // left amplitudes of the bra (L_i or Lambda)
  int i, j;
  double wi, R0j;
  PairData* P;
  double* wg = nullptr;   // metric-weighted gamma (arena)
};

static int multipliers_impl(Ctx& c, const std::vector<std::pair<int, int>>& pl, int* iters) {
  const int64_t N = c.N, nov = (int64_t)c.o * c.v, nn = (int64_t)c.n * c.n;
  const int np = (int)pl.size();
  std::vector<PairJob> jobs(np);
  for (int p = 0; p < np; ++p) {
    PairJob& J = jobs[p];
    J.i1 = pl[p].first;
    J.j1 = pl[p].second;
    J.grad_mode = (J.i1 == J.j1);
    J.has_right = (J.j1 > 0);
    J.ground_bra = (J.i1 == 0 && J.j1 > 0);
    J.i = J.i1 - 1;
    J.j = J.j1 - 1;
    J.P = &pair_of(c, J.i1, J.j1);
    J.wi = (J.i1 > 0) ? c.omega_r[J.i] : 0.0;
    J.R0j = J.has_right ? c.R0[J.j] : 1.0;
    PairData& P = *J.P;
    J.Lleft = J.ground_bra ? nullptr : (J.i1 > 0 ? c.L[J.i] : nullptr);
    if (J.grad_mode && J.has_right)
      copy_d(c, P.gamma, c.L[J.j], N);
    else if (!J.has_right)
      kc(fill(c.s, P.gamma, 0.0, N), "fill");
    else if (!J.ground_bra)
      axpby_(c, P.gamma, c.L[J.i], 1.0 / (c.omega_r[J.j] - J.wi), 0.0, N);
  }
  Arena& ar = c.eng->arena();
  int status = CC_OK;
  std::vector<int> it_z(np, 0), it_k(np, 0);
  // verbose: device time per phase
  double t_ph[6] = {0, 0, 0, 0, 0, 0};
  auto t_last = std::chrono::steady_clock::now();
  auto phase = [&](int k) {
    if (!verbose()) return;
    sync(c);
    const auto now = std::chrono::steady_clock::now();
    t_ph[k] += std::chrono::duration<double>(now - t_last).count();
    t_last = now;
  };
  {
    Tape tp(c);
    // JVP along each right state used, kept on the tape
    std::map<int, std::pair<int, int>> tanj;
    std::map<int, std::map<int, int>> tanmap;   // right state -> node -> its tangent node
    for (const PairJob& J : jobs) {
      if (!J.has_right || tanj.count(J.j)) continue;
      const int r1 = tp.G.leaf(T1of(c, c.R[J.j])), r2 = tp.G.leaf(T2of(c, c.R[J.j]));
      auto tan = tp.G.jvp({{tp.r.t1, r1}, {tp.r.t2, r2}}, tp.r.first);
      tanj[J.j] = {tan.at(tp.r.om1), tan.at(tp.r.om2)};
      tanmap[J.j] = tan;
    }
    phase(0);
    ArenaScope sc(ar);
    double* tmp = ar.alloc(N);
    // Lambda of the ground-state bra: A^T Lambda = -eta, eta = dE0/dt
    bool need_lam = false;
    for (const PairJob& J : jobs) need_lam = need_lam || J.ground_bra;
    if (need_lam && !c.have_lam) {
      if (!c.Lam) c.Lam = palloc(c, N);
      ArenaScope s2(ar);
      double* b = ar.alloc(N);
      {
        Graph Ge(*c.eng);
        EnergyNodes en = energy_graph(Ge, c, T1of(c, c.t), T2of(c, c.t));
        double* one = c.eng->scalar_slot(62);
        kc(fill(c.s, one, 1.0, 1), "fill");
        auto adj = Ge.vjp({{en.e, one}}, {en.t1, en.t2});
        copy_d(c, tmp, adj[en.t1].p, nov);
        copy_d(c, tmp + nov, adj[en.t2].p, N - nov);
      }
      kc(apply_metric(c.s, b, tmp, c.o, c.v, 1), "metric");
      axpby_(c, b, b, -1.0, 0.0, N);
      auto T = [&](const double* x, double* y, int kk) { tp.left_block(x, y, kk); };
      auto pre = [&](double* y, const double* x) {
        kc(apply_denominator(c.s, y, x, tp.deps, c.o, c.v, 0.0, 0), "precondition");
      };
      int itl = 0;
      const int st = linsolve_block(c, N, true, 1, T, pre, b, c.Lam, c.opts.tol_mult, c.opts.maxit, &itl,
                                    mixed(c));
      if (st != CC_OK) status = st;
      c.have_lam = (st == CC_OK);
    }
    for (PairJob& J : jobs)
      if (J.ground_bra) {
        J.Lleft = c.Lam;
        axpby_(c, J.P->gamma, c.Lam, 1.0 / c.omega_r[J.j], 0.0, N);
      }
    for (PairJob& J : jobs) {
      PairData& P = *J.P;
      J.wg = ar.alloc(N);
      kc(apply_metric(c.s, J.wg, P.gamma, c.o, c.v, 0), "metric");
      // F-matrix term: d/dt [gamma . A(t) R_j]
      if (J.has_right) {
        ArenaScope s2(ar);
        const auto& tj = tanj.at(J.j);
        auto adj = tp.G.vjp({{tj.first, J.wg}, {tj.second, J.wg + nov}}, {tp.r.t1, tp.r.t2});
        copy_d(c, tmp, adj[tp.r.t1].p, nov);
        copy_d(c, tmp + nov, adj[tp.r.t2].p, N - nov);
        kc(apply_metric(c.s, P.eta_t, tmp, c.o, c.v, 1), "metric");
      } else {
        kc(fill(c.s, P.eta_t, 0.0, N), "fill");
      }
      if (J.ground_bra) {
        // reference row: (1/omega_j) d/dt [eta(t) . R_j]
        ArenaScope s2(ar);
        EnergyTangent et(c, J.j);
        double* g0 = c.eng->scalar_slot(61);
        kc(fill(c.s, g0, 1.0 / c.omega_r[J.j], 1), "fill");
        auto adj = et.G.vjp({{et.te, g0}}, {et.en.t1, et.en.t2});
        copy_d(c, tmp, adj[et.en.t1].p, nov);
        copy_d(c, tmp + nov, adj[et.en.t2].p, N - nov);
        double* e2 = ar.alloc(N);
        kc(apply_metric(c.s, e2, tmp, c.o, c.v, 1), "metric");
        axpby_(c, P.eta_t, e2, 1.0, 1.0, N);
      }
      if (J.grad_mode) {
        // dE0/dt (packed-gradient convention), added to eta_t
        ArenaScope s2(ar);
        Graph Ge(*c.eng);
        EnergyNodes en = energy_graph(Ge, c, T1of(c, c.t), T2of(c, c.t));
        double* one = c.eng->scalar_slot(62);
        kc(fill(c.s, one, 1.0, 1), "fill");
        auto adj = Ge.vjp({{en.e, one}}, {en.t1, en.t2});
        copy_d(c, tmp, adj[en.t1].p, nov);
        copy_d(c, tmp + nov, adj[en.t2].p, N - nov);
        double* et = ar.alloc(N);
        kc(apply_metric(c.s, et, tmp, c.o, c.v, 1), "metric");
        axpby_(c, P.eta_t, et, 1.0, 1.0, N);
        kc(fill(c.s, P.dtrans, 0.0, nn), "fill");
      } else {
        // overlap term: R0_j L_i + singles s_ia = sum_jb L2_ijab R1_jb + L2_iiaa R1_ia
        ArenaScope s2(ar);
        Graph Gs(*c.eng);
        const double* sv = nullptr;
        if (J.has_right) {
          const int l2 = Gs.leaf(T2of(c, const_cast<double*>(J.Lleft))), rr1 = Gs.leaf(T1of(c, c.R[J.j]));
          const int sn = Gs.node({c.o, c.v}, {mul(1, op(l2, "ijab"), op(rr1, "jb"), "ia"),
                                              mul(1, op(l2, "iiaa"), op(rr1, "ia"), "ia")});
          sv = Gs.val(sn).p;
        }
        axpby_(c, P.eta_t, J.Lleft, J.R0j, 1.0, N);
        if (sv) axpby_(c, P.eta_t, sv, 1.0, 1.0, nov);
        // transition density D_pq = <L_i| E_pq |R_j>: seeds L_i on A R_j,
        // R0_j L_i + s on Omega (singles), wrt f
        double* wl = ar.alloc(N);
        kc(apply_metric(c.s, wl, J.Lleft, c.o, c.v, 0), "metric");
        double* sp = ar.alloc(N);
        axpby_(c, sp, wl, J.R0j, 0.0, N);
        if (sv) axpby_(c, sp, sv, 1.0, 1.0, nov);
        std::map<int, const double*> seeds{{tp.r.om1, sp}, {tp.r.om2, sp + nov}};
        if (J.has_right) {
          const auto& tj = tanj.at(J.j);
          seeds[tj.first] = wl;
          seeds[tj.second] = wl + nov;
        }
        auto adj = tp.G.vjp(seeds, {tp.r.f});
        copy_d(c, P.dtrans, adj[tp.r.f].p, nn);
        if (J.ground_bra) {
          // reference row of the bra: R0_j dE/df + d(eta . R_j)/df.  The
          // sweep above leaves out E(f) (L . R_j), which vanishes for an
          // excited bra but is -R0_j E(f) here (Lambda . R_j = -R0_j), so the
          // two energy terms cancel and only d(eta . R_j)/df remains.
          ArenaScope s3(ar);
          EnergyTangent et(c, J.j);
          double* a1 = c.eng->scalar_slot(59);
          kc(fill(c.s, a1, 1.0, 1), "fill");
          auto adje = et.G.vjp({{et.te, a1}}, {et.en.f});
          axpby_(c, P.dtrans, adje[et.en.f].p, 1.0, 1.0, nn);
        }
      }
    }
    // zeta: A^T zeta = -eta_t, closed form for (i, 0), the rest in blocks
    phase(1);
    std::vector<int> solve;
    for (int p = 0; p < np; ++p) {
      const PairJob& J = jobs[p];
      if (!J.grad_mode && !J.has_right)
        axpby_(c, J.P->zeta, c.L[J.i], -1.0 / J.wi, 0.0, N);
      else
        solve.push_back(p);
    }
    for (size_t b0 = 0; b0 < solve.size(); b0 += kMaxBlockRhs) {
      const int kb = (int)std::min<size_t>(kMaxBlockRhs, solve.size() - b0);
      ArenaScope s2(ar);
      double* Bm = ar.alloc((int64_t)kb * N);
      double* Xm = ar.alloc((int64_t)kb * N);
      for (int q = 0; q < kb; ++q) axpby_(c, Bm + (int64_t)q * N, jobs[solve[b0 + q]].P->eta_t, -1.0, 0.0, N);
      auto T = [&](const double* x, double* y, int kk) { tp.left_block(x, y, kk); };
      auto pre = [&](double* y, const double* x) {
        kc(apply_denominator(c.s, y, x, tp.deps, c.o, c.v, 0.0, 0), "precondition");
      };
      std::vector<int> its(kb, 0);
      const int st = linsolve_block(c, N, true, kb, T, pre, Bm, Xm, c.opts.tol_mult, c.opts.maxit,
                                    its.data(), mixed(c));
      if (st != CC_OK) status = st;
      for (int q = 0; q < kb; ++q) {
        copy_d(c, jobs[solve[b0 + q]].P->zeta, Xm + (int64_t)q * N, N);
        it_z[solve[b0 + q]] = its[q];
      }
    }
    // d Phi / d(f, g) with Phi = zeta.Omega + gamma.(A R_j) (+ E0)
    phase(2);
    for (PairJob& J : jobs) {
      PairData& P = *J.P;
      ArenaScope s2(ar);
      double* wz = ar.alloc(N);
      kc(apply_metric(c.s, wz, P.zeta, c.o, c.v, 0), "metric");
      std::map<int, const double*> seeds{{tp.r.om1, wz}, {tp.r.om2, wz + nov}};
      if (J.has_right) {
        const auto& tj = tanj.at(J.j);
        seeds[tj.first] = J.wg;
        seeds[tj.second] = J.wg + nov;
      }
      // adjoints of the leaves and of every integral use, primal and (along
      // R_j) tangent
      std::vector<int> wrt{tp.r.f, tp.r.bl, tp.r.br, tp.r.wov, tp.r.gov};
      std::vector<int> tuse(NUSE, -1);
      for (int u = 0; u < NUSE; ++u) wrt.push_back(tp.r.use[u]);
      if (J.has_right) {
        const auto& tm = tanmap.at(J.j);
        for (int u = 0; u < NUSE; ++u) {
          auto it = tm.find(tp.r.use[u]);
          if (it != tm.end()) {
            tuse[u] = it->second;
            wrt.push_back(tuse[u]);
          }
        }
      }
      auto adj = tp.G.vjp(seeds, wrt);
      copy_d(c, P.Fbar, adj[tp.r.f].p, nn);
      const int64_t v3o = (int64_t)c.v * c.v * c.v * c.o, o2v2 = (int64_t)c.o * c.o * c.v * c.v,
                    nB = (int64_t)c.naux * nn;
      // vvvv factors: the seeds of the doubles residual and of its tangent
      if (!P.ylad) P.ylad = palloc(c, 2 * o2v2);
      copy_d(c, P.ylad, wz + nov, o2v2);
      P.nlad = 1;
      P.jr = -1;
      if (J.has_right) {
        copy_d(c, P.ylad + o2v2, J.wg + nov, o2v2);
        P.nlad = 2;
        P.jr = J.j;
      }
      if (!P.gWov) P.gWov = palloc(c, v3o);
      if (!P.gGov) P.gGov = palloc(c, o2v2);
      if (!P.Bbar) P.Bbar = palloc(c, nB);
      copy_d(c, P.gWov, adj[tp.r.wov].p, v3o);
      copy_d(c, P.gGov, adj[tp.r.gov].p, o2v2);
      copy_d(c, P.Bbar, adj[tp.r.bl].p, nB);
      axpby_(c, P.Bbar, adj[tp.r.br].p, 1.0, 1.0, nB);
      for (int u = 0; u < NUSE; ++u) {
        const Tensor& a = adj[tp.r.use[u]];
        if (!P.guse[u]) P.guse[u] = palloc(c, a.size());
        copy_d(c, P.guse[u], a.p, a.size());
        if (tuse[u] >= 0) {
          const Tensor& at = adj[tuse[u]];
          if (!P.guse_t[u]) P.guse_t[u] = palloc(c, at.size());
          copy_d(c, P.guse_t[u], at.p, at.size());
        }
      }
      P.has_tan = J.has_right;
      P.hf_term = false;
      if (J.grad_mode) {
        // + dE0/d(f, g): correlation energy by the energy graph (f and the
        // bare (ia|jb) block), E_HF = 2 sum_i f_ii - sum_ij (2 g_iijj - g_ijji):
        // its f part here, its two-electron part where the factor enters
        Graph Ge(*c.eng);
        EnergyNodes en = energy_graph(Ge, c, T1of(c, c.t), T2of(c, c.t));
        double* one = c.eng->scalar_slot(62);
        kc(fill(c.s, one, 1.0, 1), "fill");
        auto adje = Ge.vjp({{en.e, one}}, {en.f, en.gov});
        axpby_(c, P.Fbar, adje[en.f].p, 1.0, 1.0, nn);
        axpby_(c, P.gGov, adje[en.gov].p, 1.0, 1.0, o2v2);
        const int64_t oo = (int64_t)c.o;
        hipLaunchKernelGGL(diag_occ_add_kernel, dim3((unsigned)((oo + 255) / 256)), dim3(256), 0, c.s,
                           P.Fbar, (int64_t)c.n, c.o, 2.0);
        hip_check(hipGetLastError(), "HF energy terms");
        P.hf_term = true;
      }
      if (J.ground_bra) {
        // reference row: (1/omega_j) eta(t; f, g) . R_j through f and (kc|ld)
        EnergyTangent et(c, J.j);
        double* g0 = c.eng->scalar_slot(61);
        kc(fill(c.s, g0, 1.0 / c.omega_r[J.j], 1), "fill");
        auto adje = et.G.vjp({{et.te, g0}}, {et.en.f, et.en.gov});
        axpby_(c, P.Fbar, adje[et.en.f].p, 1.0, 1.0, nn);
        axpby_(c, P.gGov, adje[et.en.gov].p, 1.0, 1.0, o2v2);
      }
      // the bare blocks are products of the factor: fold their adjoints into
      // d Phi / d B (for the orbital-rotation derivative)
      fold_bare_adjoints(c, P);
    }
  }
  phase(3);
  if (!c.opts.relaxed) {
    for (PairJob& J : jobs) {
      kc(fill(c.s, J.P->kbar, 0.0, nov), "fill");
      kc(fill(c.s, J.P->eta_k, 0.0, nov), "fill");
    }
  } else {
    ArenaScope sc(ar);
    double* k0 = ar.alloc(nov);
    kc(fill(c.s, k0, 0.0, nov), "fill");
    Graph G(*c.eng);
    RotNodes rn = rotation_graph(G, c, tview(k0, {c.o, c.v}));
    double* b = ar.alloc(nov);
    double* seed = ar.alloc(nn);
    // (A^HF)^T x, A^HF_(ai),(bj) = dF_ai/dkappa_bj
    auto T = [&](const double* x, double* y) {
      ArenaScope s2(ar);
      kc(fill(c.s, seed, 0.0, nn), "fill");
      ViewSpec vs;  // seed[o+a][i] = x[i][a]
      vs.nd = 2;
      vs.dims[0] = c.o; vs.dims[1] = c.v;
      vs.ostr[0] = 1; vs.ostr[1] = c.n;
      vs.obase = (int64_t)c.o * c.n;
      vs.istr[0] = c.v; vs.istr[1] = 1;
      kc(view_gather(c.s, seed, x, vs, 1.0, 0.0), "embed");
      auto adj = G.vjp({{rn.fr, seed}}, {rn.kap});
      copy_d(c, y, adj[rn.kap].p, nov);
    };
    // preconditioner: orbital-energy differences on the singles block
    auto pre1 = [&](double* y, const double* x) {
      ArenaScope s3(ar);
      double* big = ar.alloc(N);
      kc(fill(c.s, big, 0.0, N), "fill");
      copy_d(c, big, x, nov);
      kc(apply_denominator(c.s, big, big, c.eps.p, c.o, c.v, 0.0, 0), "precondition");
      copy_d(c, y, big, nov);
    };
    for (int p = 0; p < np; ++p) {
      const PairJob& J = jobs[p];
      PairData& P = *J.P;
      // eta_kappa = -(D_ai - D_ia) + d/dkappa Phi
      {
        ArenaScope s2(ar);
        auto adj = G.vjp({{rn.fr, P.Fbar}, {rn.db, P.Bbar}}, {rn.kap});
        copy_d(c, P.eta_k, adj[rn.kap].p, nov);
      }
      if (!J.grad_mode) {
        ArenaScope s2(ar);
        Graph Gd(*c.eng);
        const int d = Gd.leaf(tview(P.dtrans, {c.n, c.n}));
        const Range O{0, c.o}, V{c.o, c.v};
        const int e1 = Gd.node({c.o, c.v}, {lin(-1, op(d, "ai", {V, O}), "ia"), lin(1, op(d, "ia", {O, V}), "ia")});
        axpby_(c, P.eta_k, Gd.val(e1).p, 1.0, 1.0, nov);
      }
      phase(4);
      // (A^HF)^T kappa_bar = -eta_kappa (eq. orbitalrelax)
      axpby_(c, b, P.eta_k, -1.0, 0.0, nov);
      const int st = linsolve_refined(c, nov, false, T, pre1, b, P.kbar, c.opts.tol_mult, c.opts.maxit,
                                      &it_k[p]);
      if (st != CC_OK) status = st;
      phase(5);
    }
  }
  if (verbose())
    std::fprintf(stderr,
                 "[multipliers] %d pairs: tape+jvp %.3f rhs %.3f zeta %.3f dens-adjoint %.3f eta-kappa %.3f "
                 "kappa %.3f s\n", np, t_ph[0], t_ph[1], t_ph[2], t_ph[3], t_ph[4], t_ph[5]);
  for (PairJob& J : jobs) {
    J.P->have_mult = true;
    J.P->have_dens = false;
  }
  if (iters)
    for (int p = 0; p < np; ++p) {
      iters[2 * p] = it_z[p];
      iters[2 * p + 1] = it_k[p];
    }
  sync(c);
  return status;
}

// One-sided blocks of the two-electron density (Sec. II C, eq.
// NAC_NC_densities).  A use sum_P a(B)[P] (x) b(B)[P] enters the coupling of
// a direction as sum_P <Gbar, a(dB)[P] (x) b(dB)[P]> with a, b linear in the
// factor (T1-transformed blocks, their forward derivatives along R1_j, or
// bare blocks).  Its adjoint Gbar is lifted through the transform of one
// half (a reverse sweep over the factor graph with the other half's entries
// as the batch), which turns it into one linear form on the symmetric pairs
// of the bare factor per entry of the other half; the other half stays the
// direction's own transformed block.  The bare (kc|bd) and (kc|ld) blocks
// enter with the identity as their lifted half.
static void lift_uses(Ctx& c, PairData& P) {
  const int64_t o = c.o, v = c.v, n = c.n, nn = n * n, m = n * (n + 1) / 2;
  const bool tn = P.has_tan;
  const int64_t len[NGRP] = {v * o, tn ? v * o : 0, o * o, tn ? o * o : 0, o * v};
  int64_t cols = 0;
  for (int g = 0; g < NGRP; ++g) {
    P.goff[g] = cols;
    P.glen[g] = len[g];
    cols += len[g];
  }
  if (!P.gam || P.gcols != cols) P.gam = palloc(c, cols * m);
  P.gcols = cols;
  Arena& ar = c.eng->arena();
  const int64_t shape_of[NUSE][4] = {{v, o, v, o}, {o, o, o, o}, {o, o, v, v}, {v, o, o, v},
                                     {v, v, o, v}, {v, v, o, o}, {o, o, o, v}, {n, n, 1, 1}};
  for (int g = 0; g < NGRP; ++g) {
    if (!len[g]) continue;
    // the operand entry is a pair (lead, inner); batches of whole leads
    const int64_t lead = (g == G_VO || g == G_VOT) ? v : o, inner = len[g] / lead;
    const int64_t budget = (int64_t)1 << 27;   // doubles of lifted rows per batch
    const int64_t cl = std::max<int64_t>(1, std::min<int64_t>(lead, budget / (inner * nn)));
    for (int64_t l0 = 0; l0 < lead; l0 += cl) {
      const int64_t lc = std::min(cl, lead - l0), rows = lc * inner;
      ArenaScope sc(ar);
      Graph G(*c.eng);
      double* zb = ar.alloc(rows * nn);
      kc(fill(c.s, zb, 0.0, rows * nn), "fill");
      const int t1 = G.leaf(T1of(c, c.t));
      const int b = G.leaf(tview(zb, {rows, n, n}));
      const int first = G.size();
      const FactorNodes F = factor_graph(G, c, t1, b);
      std::map<int, int> tm;
      if (tn) {
        const int r1 = G.leaf(T1of(c, c.R[P.jr]));
        tm = G.jvp({{t1, r1}}, first);
      }
      // seed terms per lifted node: the use adjoint with the operand's pair
      // first (its lead index restricted to this batch)
      std::map<int, std::vector<Term>> terms;
      std::map<int, std::vector<int64_t>> shapes;
      auto add = [&](int target, int u, bool tangent, const char* lin_, char leadlab, const char* lout) {
        double* src = tangent ? P.guse_t[u] : P.guse[u];
        if (!src) return;
        const std::vector<int64_t> sh(shape_of[u], shape_of[u] + 4);
        const int gl = G.leaf(tview(src, sh));
        std::vector<Range> box;
        for (int k = 0; k < 4; ++k) box.push_back(lin_[k] == leadlab ? Range{l0, lc} : Range{0, sh[k]});
        std::vector<int64_t> osh;
        for (int k = 0; k < 4; ++k) {
          const int pos = (int)(std::string(lin_).find(lout[k]));
          osh.push_back(lout[k] == leadlab ? lc : sh[pos]);
        }
        terms[target].push_back(lin(1, op(gl, lin_, box), lout));
        shapes[target] = osh;
      };
      auto T = [&](int node) { return tm.count(node) ? tm.at(node) : -1; };
      switch (g) {
        case G_VO:
          add(F.vo, U_VOVO, false, "aibj", 'b', "bjai");
          if (tn) add(T(F.vo), U_VOVO, true, "aibj", 'b', "bjai");
          break;
        case G_VOT:
          add(F.vo, U_VOVO, true, "aibj", 'b', "bjai");
          break;
        case G_OO:
          add(F.oo, U_OOOO, false, "kilj", 'l', "ljki");
          add(F.vv, U_OOVV, false, "kiac", 'k', "kiac");
          add(F.vv, U_VVOO, false, "acki", 'k', "kiac");
          if (tn) {
            add(T(F.oo), U_OOOO, true, "kilj", 'l', "ljki");
            add(T(F.vv), U_OOVV, true, "kiac", 'k', "kiac");
            add(T(F.vv), U_VVOO, true, "acki", 'k', "kiac");
          }
          break;
        case G_OOT:
          add(F.oo, U_OOOO, true, "kilj", 'l', "ljki");
          add(F.vv, U_OOVV, true, "kiac", 'k', "kiac");
          add(F.vv, U_VVOO, true, "acki", 'k', "kiac");
          break;
        default:  // G_OV
          add(F.vo, U_VOOV, false, "aikc", 'k', "kcai");
          add(F.vv, U_VVOV, false, "adkc", 'k', "kcad");
          add(F.oo, U_OOOV, false, "kilc", 'l', "lcki");
          if (tn) {
            add(T(F.vo), U_VOOV, true, "aikc", 'k', "kcai");
            add(T(F.vv), U_VVOV, true, "adkc", 'k', "kcad");
            add(T(F.oo), U_OOOV, true, "kilc", 'l', "lcki");
          }
          break;
      }
      std::map<int, const double*> seeds;
      for (auto& kv : terms) {
        if (kv.first < 0) throw Error(-3, "density lift: missing tangent node");
        seeds[kv.first] = G.val(G.node(shapes.at(kv.first), kv.second)).p;
      }
      auto adj = G.vjp(seeds, {b});
      double* bb = adj.at(b).p;
      if (g == G_OV) {
        // (kc|bd): bb[(k, c)][o + b][o + d] += dPhi/dWov[c][d][k][b]
        const int gw = G.leaf(tview(P.gWov, {v, v, o, v}));
        const int pw = G.node({lc, v, v, v}, {lin(1, op(gw, "cdkb", {{0, v}, {0, v}, {l0, lc}, {0, v}}), "kcbd")});
        ViewSpec vs;
        vs.nd = 3;
        vs.dims[0] = rows; vs.dims[1] = v; vs.dims[2] = v;
        vs.ostr[0] = nn; vs.ostr[1] = n; vs.ostr[2] = 1;
        vs.obase = o * n + o;
        vs.istr[0] = v * v; vs.istr[1] = v; vs.istr[2] = 1;
        kc(view_gather(c.s, bb, G.val(pw).p, vs, 1.0, 1.0), "bare vvov");
        // (kc|ld): bb[(k, c)][l][o + d] += dPhi/dGov[k][c][l][d]
        ViewSpec vg;
        vg.nd = 3;
        vg.dims[0] = rows; vg.dims[1] = o; vg.dims[2] = v;
        vg.ostr[0] = nn; vg.ostr[1] = n; vg.ostr[2] = 1;
        vg.obase = o;
        vg.istr[0] = o * v; vg.istr[1] = v; vg.istr[2] = 1;
        vg.ibase = l0 * v * o * v;
        kc(view_gather(c.s, bb, P.gGov, vg, 1.0, 1.0), "bare ovov");
      }
      kc(pack_pairs(c.s, P.gam + (P.goff[g] + l0 * inner) * m, m, bb, nn, rows, c.o, c.v, true),
         "pair packing");
    }
  }
}

// D_eff = dPhi/df + kappa-bar embedded in the vo block (Sec. II C); the
// two-electron density as one-sided blocks (lift_uses) and the factorised
// vvvv block.
static void densities_impl(Ctx& c, int i1, int j1) {
  PairData& P = c.pairs.at({i1, j1});
  const int64_t nn = (int64_t)c.n * c.n;
  copy_d(c, P.Deff, P.Fbar, nn);
  ViewSpec vs;  // Deff[o+a][i] += kbar[i][a]
  vs.nd = 2;
  vs.dims[0] = c.o; vs.dims[1] = c.v;
  vs.ostr[0] = 1; vs.ostr[1] = c.n;
  vs.obase = (int64_t)c.o * c.n;
  vs.istr[0] = c.v; vs.istr[1] = 1;
  kc(view_gather(c.s, P.Deff, P.kbar, vs, 1.0, 1.0), "kappa embed");
  lift_uses(c, P);
  P.have_dens = true;
}

// F^q = sum D_eff dh^q + sum Gamma dg^q with dg^q = sum_P dB^q[P] (x) dB^q[P]
// (Sec. II C, eq. NAC_NC): every place the integrals enter the Lagrangian is
// bilinear in the factor, so the second term is a sum over P of quadratic
// forms in the direction's factor dB^q[P].  All directions of a batch go
// through each step together, with the rows (q, P) as one index:
//  * one-sided blocks: x = packed pairs of dB^q[P], Z = x gam^T (one GEMM),
//    contracted row by row with the direction's transformed operands;
//  * vvvv: the factorised block formed once per call, packed over symmetric
//    pairs, then x_vv Gw^T x_vv;
//  * the Fock matrix's dependence on g through D_eff (2 J - K of dg), the
//    Fock correction of the T1 transform and, for the energy Lagrangian,
//    E_HF's two-electron part, as small contractions per row.
static void nacme_impl(Ctx& c, int i1, int j1, int nq, const double* dh, const double* dB,
                       double* F) {
  PairData& P = c.pairs.at({i1, j1});
  const int64_t o = c.o, v = c.v, n = c.n, nn = n * n, Pn = c.naux, m = n * (n + 1) / 2;
  const int64_t mv = v * (v + 1) / 2, xvv = o * (o + 1) / 2 + o * v, gc = P.gcols;
  const bool tn = P.has_tan;
  Arena& ar = c.eng->arena();
  ArenaScope sc(ar);
  // packed vvvv block from its factors, a chunk of rows c at a time: the
  // chunk's rows of d Phi/dW (M1) and its columns c (M2, the image with the
  // first and third indices swapped), two GEMMs over the o^2 pairs each
  double* Gw = ar.alloc(mv * mv);
  {
    const int64_t cch = vvvv_chunk(c), v2 = v * v, o2v2 = o * o * v2;
    ArenaScope s2(ar);
    double* M1 = ar.alloc(cch * v * v2);
    double* M2 = ar.alloc(cch * v * v2);
    const double* Xf[2] = {c.t + o * v, P.nlad > 1 ? c.R[P.jr] + o * v : nullptr};
    const double* Yf[2] = {P.ylad, P.ylad + o2v2};
    for (int64_t c0 = 0; c0 < v; c0 += cch) {
      const int cc = (int)std::min(cch, v - c0);
      for (int f = 0; f < P.nlad; ++f) {
        const double beta = f == 0 ? 0.0 : 1.0;
        kc(gemm_f64(c.s, true, false, (int)(cc * v), (int)v2, (int)(o * o), 1, 1.0, Xf[f] + c0 * v, v2, 0,
                    Yf[f], v2, 0, beta, M1, v2, 0), "vvvv rows");
        kc(gemm_f64(c.s, true, false, (int)v2, (int)(cc * v), (int)(o * o), 1, 1.0, Xf[f], v2, 0,
                    Yf[f] + c0 * v, v2, 0, beta, M2, cc * v, 0), "vvvv columns");
      }
      kc(pack_vvvv_rows(c.s, Gw, M1, M2, c.v, (int)c0, cc), "vvvv packing");
    }
  }
  // directions per batch from the arena use of one direction's rows
  // (the mixed modes add fp32 packings of the pair rows: half a double each)
  const int64_t per_dir = Pn * (m + 2 * gc + mv + (m + mv) / 2 + 3 * (n * o + o * o + v * o) + n * v +
                                4 * n * o + 2 * o * o);
  const int64_t budget = (int64_t)2 << 30;   // doubles
  const int kq = (int)std::max<int64_t>(1, std::min<int64_t>(nq, budget / per_dir));
  double* f1 = ar.alloc(kq);
  std::vector<double> sh, fh(kq);
  for (int q0 = 0; q0 < nq; q0 += kq) {
    const int nb = std::min(kq, nq - q0);
    const int64_t R = nb * Pn;
    ArenaScope s2(ar);
    double* db_p = const_cast<double*>(dB) + (int64_t)q0 * Pn * nn;
    double* x = ar.alloc(R * m);
    kc(pack_pairs(c.s, x, m, db_p, nn, R, c.o, c.v, false), "pair packing");
    double* s = ar.alloc(R);
    double* Bop = ar.alloc(R * gc);
    Graph G(*c.eng);
    const Range AP{0, R}, O{0, o}, A{0, n}, Ol{0, o};
    // the two products over packed pairs (one-sided blocks and vvvv),
    // Z[r][y] = sum_k x[r][kb + k] Y[y][k]: fp64 in the fp64 mode, fp32
    // operands (fp32 accumulation, fp64 result) in the mixed modes, as the
    // solvers' large contractions
    const int xl = G.leaf(tview(x, {R, m}));
    auto pair_product = [&](double* Y, int64_t cols, Range kb) -> const double* {
      if (!mixed(c)) {
        double* z = ar.alloc(R * cols);
        kc(gemm_f64(c.s, false, true, (int)R, (int)cols, (int)kb.len, 1, 1.0, x + kb.lo, m, 0, Y, kb.len, 0,
                    0.0, z, cols, 0),
           "pair product");
        return z;
      }
      c.eng->set_lowp(true);
      c.eng->set_bf16(false);
      const int yl = G.leaf(tview(Y, {cols, kb.len}));
      const int z = G.node({R, cols}, {mul(1, op(xl, "rk", {AP, kb}), op(yl, "yk"), "ry")});
      c.eng->set_lowp(false);
      return G.val(z).p;
    };
    const double* Z = pair_product(P.gam, gc, Range{0, m});
    const int t1 = G.leaf(T1of(c, c.t));
    const int db = G.leaf(tview(db_p, {R, n, n}));
    const int first = G.size();
    const FactorNodes Fd = factor_graph(G, c, t1, db, false);
    std::map<int, int> tm;
    if (tn) {
      const int r1 = G.leaf(T1of(c, c.R[P.jr]));
      tm = G.jvp({{t1, r1}}, first);
    }
    copy_rows(c, Bop + P.goff[G_VO], gc, G.val(Fd.vo).p, v * o, v * o, R);
    copy_rows(c, Bop + P.goff[G_OO], gc, G.val(Fd.oo).p, o * o, o * o, R);
    if (tn) {
      copy_rows(c, Bop + P.goff[G_VOT], gc, G.val(tm.at(Fd.vo)).p, v * o, v * o, R);
      copy_rows(c, Bop + P.goff[G_OOT], gc, G.val(tm.at(Fd.oo)).p, o * o, o * o, R);
    }
    {
      ViewSpec vs;  // Bop[r][ov + k v + c] = dB[r][k][o + c]
      vs.nd = 3;
      vs.dims[0] = R; vs.dims[1] = o; vs.dims[2] = v;
      vs.ostr[0] = gc; vs.ostr[1] = v; vs.ostr[2] = 1;
      vs.obase = P.goff[G_OV];
      vs.istr[0] = nn; vs.istr[1] = n; vs.istr[2] = 1;
      vs.ibase = o;
      kc(view_gather(c.s, Bop, db_p, vs, 1.0, 0.0), "ov block");
    }
    kc(rowdot(c.s, s, Z, gc, Bop, gc, R, gc, 1.0, 0.0), "row dots");
    // vvvv
    const double* Zw = pair_product(Gw, mv, Range{xvv, mv});
    kc(rowdot(c.s, s, Zw, mv, x + xvv, m, R, mv, 1.0, 1.0), "row dots");
    // Fock correction 2 sum_P tr(D[P]) B[P] - sum_P D[P] B[P][occ rows]
    auto fcorr_rows = [&](const double* gbar, int dnode) {
      const int fc = G.leaf(tview(const_cast<double*>(gbar), {n, n}));
      const int y = G.node({R}, {mul(1, op(fc, "pq"), op(db, "Ppq"), "P")});
      const int trd = G.node({R}, {lin(1, op(dnode, "Pkk", {AP, O, Ol}), "P")});
      kc(rowdot(c.s, s, G.val(trd).p, 1, G.val(y).p, 1, R, 1, 2.0, 1.0), "row dots");
      const int zk = G.node({R, n, o}, {mul(1, op(fc, "pq"), op(db, "Pkq", {AP, O, A}), "Ppk")});
      kc(rowdot(c.s, s, G.val(dnode).p, n * o, G.val(zk).p, n * o, R, n * o, -1.0, 1.0), "row dots");
    };
    fcorr_rows(P.guse[U_FCORR], Fd.d);
    if (tn && P.guse_t[U_FCORR] && tm.count(Fd.d)) fcorr_rows(P.guse_t[U_FCORR], tm.at(Fd.d));
    // the Fock matrix's dependence on g: 2 D_eff.J(dg) - D_eff.K(dg)
    const int de = G.leaf(tview(P.Deff, {n, n}));
    const int sn = G.node({R}, {lin(1, op(db, "Pkk", {AP, O, O}), "P")});
    const int yd = G.node({R}, {mul(1, op(de, "pq"), op(db, "Ppq"), "P")});
    kc(rowdot(c.s, s, G.val(sn).p, 1, G.val(yd).p, 1, R, 1, 2.0, 1.0), "row dots");
    const int zd = G.node({R, n, o}, {mul(1, op(de, "pq"), op(db, "Pkq", {AP, O, A}), "Ppk")});
    const int dpk = G.node({R, n, o}, {lin(1, op(db, "Ppk", {AP, A, O}), "Ppk")});
    kc(rowdot(c.s, s, G.val(dpk).p, n * o, G.val(zd).p, n * o, R, n * o, -1.0, 1.0), "row dots");
    // E_HF two-electron part: -sum_ij (2 dg_iijj - dg_ijji)
    if (P.hf_term) {
      kc(rowdot(c.s, s, G.val(sn).p, 1, G.val(sn).p, 1, R, 1, -2.0, 1.0), "row dots");
      const int d1 = G.node({R, o, o}, {lin(1, op(db, "Pij", {AP, O, O}), "Pij")});
      const int d2 = G.node({R, o, o}, {lin(1, op(db, "Pji", {AP, O, O}), "Pij")});
      kc(rowdot(c.s, s, G.val(d1).p, o * o, G.val(d2).p, o * o, R, o * o, 1.0, 1.0), "row dots");
    }
    kc(rowdot(c.s, f1, dh + (int64_t)q0 * nn, nn, P.Deff, 0, nb, nn, 1.0, 0.0), "row dots");
    sh.resize(R);
    hip_check(hipMemcpyAsync(sh.data(), s, R * sizeof(double), hipMemcpyDeviceToHost, c.s), "copy D2H");
    hip_check(hipMemcpyAsync(fh.data(), f1, nb * sizeof(double), hipMemcpyDeviceToHost, c.s), "copy D2H");
    sync(c);
    for (int q = 0; q < nb; ++q) {
      double f2 = 0.0;
      for (int64_t p = 0; p < Pn; ++p) f2 += sh[q * Pn + p];
      F[q0 + q] = fh[q] + f2;
    }
  }
}

}  // namespace nm

// ======================================================================= ABI
using nm::Ctx;
using nm::Error;

static int fail(Ctx* c, const Error& e) {
  if (c) {
    c->err = e.what();
    if (e.code == CC_ERR_HIP) c->sticky = true;
  }
  return e.code;
}

#define ABI_GUARD(c)                                                   \
  if (!(c)) return CC_ERR_ARG;                                         \
  if ((c)->sticky) {                                                   \
    (c)->err = "context unusable after an earlier device failure";     \
    return CC_ERR_HIP;                                                 \
  }

extern "C" {

void cc_default_opts(cc_opts* o) {
  if (!o) return;
  o->precision = CC_FP64;
  o->relaxed = 1;
  o->tol_ground = 1e-10;
  o->tol_eom = 1e-9;
  o->tol_mult = 1e-9;
  o->maxit = 200;
  o->diis_dim = 8;
  o->davidson_block = 2;
  o->davidson_max = 120;
  o->mixed_min_flops = 1e9;
}

const char* nm_version(void) { return "nacme-mi355x 0.1 (gfx950, fp64)"; }

int cc_create(cc_ctx** out, int o, int v, int naux, const double* eps, const double* B,
              const cc_opts* opts, void* stream) {
  if (!out || o < 1 || v < 1 || naux < 1 || !eps || !B) return CC_ERR_ARG;
  *out = nullptr;
  Ctx* c = new Ctx();
  try {
    c->o = o;
    c->v = v;
    c->n = o + v;
    c->naux = naux;
    const int64_t nov = (int64_t)o * v;
    c->N = nov + nov * nov;
    if (opts) c->opts = *opts; else cc_default_opts(&c->opts);
    if (c->opts.precision != CC_FP64 && c->opts.precision != CC_FP32_REFINE &&
        c->opts.precision != CC_BF16X3_REFINE)
      throw Error(CC_ERR_ARG, "unknown precision mode");
    c->s = (hipStream_t)stream;
    c->eng.reset(new nm::Engine(c->s));
    c->eng->set_lowp_min_flops(c->opts.mixed_min_flops);
    const int64_t n = c->n, nn = n * n;
    c->eps = nm::tview(nm::palloc(*c, n), {n});
    nm::copy_d(*c, c->eps.p, eps, n);
    c->eps_h.resize(n);
    nm::hip_check(hipMemcpyAsync(c->eps_h.data(), eps, n * sizeof(double), hipMemcpyDeviceToHost, c->s), "D2H");
    nm::sync(*c);
    for (int k = 0; k < n; ++k)
      if (!std::isfinite(c->eps_h[k])) throw Error(CC_ERR_ARG, "non-finite orbital energy");
    for (int i = 0; i < o; ++i)
      for (int a = 0; a < v; ++a)
        if (!(c->eps_h[o + a] > c->eps_h[i])) throw Error(CC_ERR_ARG, "virtual orbital energy below an occupied one");
    // f = diag(eps)
    c->f = nm::tview(nm::palloc(*c, nn), {n, n});
    nm::kc(nm::fill(c->s, c->f.p, 0.0, nn), "fill");
    {
      nm::ViewSpec vs;
      vs.nd = 1;
      vs.dims[0] = n;
      vs.ostr[0] = n + 1;
      vs.istr[0] = 1;
      nm::kc(nm::view_gather(c->s, c->f.p, c->eps.p, vs, 1.0, 0.0), "diag");
    }
    // the factor (kept) and the bare blocks the residual uses directly:
    // W[c][d][a][b] = (ac|bd), Wov[c][d][k][b] = (kc|bd), Gov[k][c][l][d] = (kc|ld),
    // each one GEMM over P
    c->B = nm::tview(nm::palloc(*c, (int64_t)naux * nn), {naux, n, n});
    nm::copy_d(*c, c->B.p, B, (int64_t)naux * nn);
    {
      const int64_t vv = (int64_t)v * v;
      c->W = nm::tview(nm::palloc(*c, vv * vv), {v, v, v, v});
      c->Wov = nm::tview(nm::palloc(*c, vv * v * o), {v, v, o, v});
      c->Gov = nm::tview(nm::palloc(*c, (int64_t)o * v * o * v), {o, v, o, v});
      nm::Graph G(*c->eng);
      const int bl = G.leaf(c->B);
      const nm::Range Oo{0, o}, Vv{o, v}, AP{0, naux};
      c->eng->contract(1.0, G.view(nm::op(bl, "Pac", {AP, Vv, Vv})), G.view(nm::op(bl, "Pbd", {AP, Vv, Vv})),
                       nm::full_view(c->W, "cdab"), true);
      c->eng->contract(1.0, G.view(nm::op(bl, "Pkc", {AP, Oo, Vv})), G.view(nm::op(bl, "Pbd", {AP, Vv, Vv})),
                       nm::full_view(c->Wov, "cdkb"), true);
      c->eng->contract(1.0, G.view(nm::op(bl, "Pkc", {AP, Oo, Vv})), G.view(nm::op(bl, "Pld", {AP, Oo, Vv})),
                       nm::full_view(c->Gov, "kcld"), true);
      // W[cd][ab] = (ac|bd) = (ca|db) = W[ab][cd] for real orbitals and a
      // factor symmetric in p, q
      c->W.pair_sym = true;
      c->W.constant = c->Wov.constant = c->Gov.constant = c->B.constant = true;
    }
    c->t = nm::palloc(*c, c->N);
    nm::kc(nm::fill(c->s, c->t, 0.0, c->N), "fill");
    c->rows_part = nm::palloc(*c, nm::rows_scratch_doubles());
    nm::sync(*c);
    *out = c;
    return CC_OK;
  } catch (const Error& e) {
    int code = e.code;
    delete c;
    return code;
  } catch (const std::exception& e) {
    delete c;
    return CC_ERR_HIP;
  }
}

void cc_destroy(cc_ctx* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  c->eng.reset();
  for (void* p : c->owned) (void)hipFree(p);
  delete c;
}

const char* cc_last_error(const cc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int cc_ground(cc_ctx* c, double* e_corr, int* iters) {
  ABI_GUARD(c);
  try {
    int st = nm::ground(*c, e_corr, iters);
    c->stage = 1;
    c->have_guess = false;
    c->have_right = c->have_left = c->gauged = false;
    c->pairs.clear();
    c->have_lam = false;
    if (st == CC_NOT_CONVERGED) c->err = "CCSD amplitudes not converged";
    return st;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int eom_solve(cc_ctx* c, int side, int nroots, double* omega, int* iters) {
  ABI_GUARD(c);
  if (c->stage < 1) { c->err = "eom_solve before cc_ground"; return CC_ERR_STATE; }
  if (side < 1 || side > 3 || nroots < 1 || nroots > (int)std::min<int64_t>(c->N, 64)) {
    c->err = "bad side or nroots";
    return CC_ERR_ARG;
  }
  try {
    // stages differ in their large work buffers: release the arena chunks
    // the previous stage left unused before this one allocates its own
    c->eng->arena().trim();
    int st = nm::eom(*c, side, nroots, omega, iters);
    if (st == CC_ERR_COMPLEX_ROOT) c->err = "complex EOM root among the requested states";
    if (st == CC_NOT_CONVERGED) c->err = "EOM states not converged";
    return st;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int multipliers(cc_ctx* c, int npairs, const int* pairs, int* iters) {
  ABI_GUARD(c);
  if (npairs < 1 || !pairs) {
    c->err = "multipliers needs at least one pair";
    return CC_ERR_ARG;
  }
  for (int p = 0; p < npairs; ++p) {
    const int i = pairs[2 * p], j = pairs[2 * p + 1];
    if (c->stage < 1 || (!c->gauged && !(i == 0 && j == 0))) {
      c->err = "multipliers before the ground state (pair (0, 0)) or the right and left EOM states";
      return CC_ERR_STATE;
    }
  }
  std::vector<std::pair<int, int>> pl;
  for (int p = 0; p < npairs; ++p) {
    const int i = pairs[2 * p], j = pairs[2 * p + 1];
    if (i < 0 || j < 0 || i > c->nroots || j > c->nroots) {
      c->err = "pair indices must satisfy 0 <= i, j <= nroots";
      return CC_ERR_ARG;
    }
    for (const auto& q : pl)
      if (q.first == i && q.second == j) {
        c->err = "a pair appears twice in one multipliers call";
        return CC_ERR_ARG;
      }
    pl.push_back({i, j});
  }
  try {
    // stages differ in their large work buffers: release the arena chunks
    // the previous stage left unused before this one allocates its own
    c->eng->arena().trim();
    return nm::multipliers_impl(*c, pl, iters);
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int densities(cc_ctx* c, int i, int j, double* D1) {
  ABI_GUARD(c);
  auto it = c->pairs.find({i, j});
  if (it == c->pairs.end() || !it->second.have_mult) {
    c->err = "densities before multipliers of this pair";
    return CC_ERR_STATE;
  }
  try {
    // stages differ in their large work buffers: release the arena chunks
    // the previous stage left unused before this one allocates its own
    c->eng->arena().trim();
    nm::densities_impl(*c, i, j);
    if (D1) nm::copy_d(*c, D1, it->second.Deff, (int64_t)c->n * c->n);
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int nacme(cc_ctx* c, int i, int j, int nq, const double* dh, const double* dB, double* F) {
  ABI_GUARD(c);
  auto it = c->pairs.find({i, j});
  if (it == c->pairs.end() || !it->second.have_dens) {
    c->err = "nacme before densities of this pair";
    return CC_ERR_STATE;
  }
  if (nq < 0 || (nq > 0 && (!dh || !dB || !F))) {
    c->err = "bad directions";
    return CC_ERR_ARG;
  }
  try {
    // stages differ in their large work buffers: release the arena chunks
    // the previous stage left unused before this one allocates its own
    c->eng->arena().trim();
    nm::nacme_impl(*c, i, j, nq, dh, dB, F);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_apply_jacobian(cc_ctx* c, int side, const double* X, double* Y) {
  ABI_GUARD(c);
  if (c->stage < 1) { c->err = "cc_apply_jacobian before cc_ground"; return CC_ERR_STATE; }
  if (!X || !Y || (side != CC_RIGHT && side != CC_LEFT)) return CC_ERR_ARG;
  try {
    nm::Tape tp(*c);
    if (side == CC_RIGHT) tp.right(X, Y); else tp.left(X, Y);
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_apply_jacobian_block(cc_ctx* c, int side, int k, const double* X, double* Y, int precision) {
  ABI_GUARD(c);
  if (c->stage < 1) { c->err = "cc_apply_jacobian_block before cc_ground"; return CC_ERR_STATE; }
  if (!X || !Y || k < 1 || (side != CC_RIGHT && side != CC_LEFT) ||
      (precision != CC_FP64 && precision != CC_FP32_REFINE && precision != CC_BF16X3_REFINE))
    return CC_ERR_ARG;
  try {
    nm::Tape tp(*c);
    c->eng->set_lowp(precision != CC_FP64);
    c->eng->set_bf16(precision == CC_BF16X3_REFINE);
    if (side == CC_RIGHT) tp.right_block(X, Y, k); else tp.left_block(X, Y, k);
    c->eng->set_lowp(false);
    c->eng->set_bf16(false);
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    c->eng->set_lowp(false);
    c->eng->set_bf16(false);
    return fail(c, e);
  }
}

int cc_residual(cc_ctx* c, const double* t, double* omega) {
  ABI_GUARD(c);
  if (!t || !omega) return CC_ERR_ARG;
  try {
    nm::ArenaScope sc(c->eng->arena());
    double* tt = c->eng->arena().alloc(c->N);
    nm::copy_d(*c, tt, t, c->N);
    nm::residual(*c, tt, omega);
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_export(cc_ctx* c, int what, int idx, int jdx, double* dst) {
  ABI_GUARD(c);
  if (!dst) return CC_ERR_ARG;
  try {
    const int64_t nn = (int64_t)c->n * c->n, nov = (int64_t)c->o * c->v;
    switch (what) {
      case CC_T: nm::copy_d(*c, dst, c->t, c->N); break;
      case CC_R:
      case CC_L:
      case CC_R0: {
        if (idx < 1 || idx > c->nroots) return CC_ERR_ARG;
        if (what == CC_R0) {
          if (!c->gauged) return CC_ERR_STATE;
          *dst = c->R0[idx - 1];
          return CC_OK;
        }
        nm::copy_d(*c, dst, (what == CC_R ? c->R : c->L)[idx - 1], c->N);
        break;
      }
      default: {
        auto it = c->pairs.find({idx, jdx});
        if (it == c->pairs.end() || !it->second.have_mult) {
          c->err = "cc_export of a pair quantity before multipliers of that pair";
          return CC_ERR_STATE;
        }
        nm::PairData& P = it->second;
        if (what == CC_ZETA) nm::copy_d(*c, dst, P.zeta, c->N);
        else if (what == CC_KAPPA) nm::copy_d(*c, dst, P.kbar, nov);
        else if (what == CC_ETA_T) nm::copy_d(*c, dst, P.eta_t, c->N);
        else if (what == CC_ETA_K) nm::copy_d(*c, dst, P.eta_k, nov);
        else if (what == CC_DTRANS) nm::copy_d(*c, dst, P.dtrans, nn);
        else if (what == CC_D1) {
          if (!P.have_dens) { c->err = "cc_export of D_eff before densities"; return CC_ERR_STATE; }
          nm::copy_d(*c, dst, P.Deff, nn);
        } else return CC_ERR_ARG;
      }
    }
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_set_guess(cc_ctx* c, int what, int idx, const double* src) {
  ABI_GUARD(c);
  if (!src || (what != CC_T && what != CC_R && what != CC_L)) return CC_ERR_ARG;
  if (what != CC_T && (idx < 1 || idx > 64)) return CC_ERR_ARG;
  try {
    if (what == CC_T) {
      nm::copy_d(*c, c->t, src, c->N);
      c->have_guess = true;
    } else {
      auto& gm = (what == CC_R) ? c->guess_R : c->guess_L;
      if (!gm.count(idx)) gm[idx] = nm::palloc(*c, c->N);
      nm::copy_d(*c, gm[idx], src, c->N);
    }
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_t2_features(cc_ctx* c, const float* mu, const float* sd, float* F) {
  ABI_GUARD(c);
  if (!F) return CC_ERR_ARG;
  try {
    nm::ArenaScope sc(c->eng->arena());
    const float* nrm = nm::feature_norm(*c, mu, sd);
    const int64_t tot = (int64_t)c->o * c->o * c->v * c->v;
    const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(nm::t2_features_kernel, dim3(g), dim3(256), 0, c->s, c->Gov.p, c->eps.p, c->o,
                       c->v, nrm, nrm + 8, F);
    nm::hip_check(hipGetLastError(), "t2 features");
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_t2_target(cc_ctx* c, float scale, float* Z) {
  ABI_GUARD(c);
  if (c->stage < 1) { c->err = "cc_t2_target before cc_ground"; return CC_ERR_STATE; }
  if (!Z || !(scale > 0.0f)) return CC_ERR_ARG;
  try {
    const int64_t tot = (int64_t)c->o * c->o * c->v * c->v, nov = (int64_t)c->o * c->v;
    const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(nm::t2_map_kernel, dim3(g), dim3(256), 0, c->s, c->Gov.p, c->eps.p, c->o, c->v,
                       c->t + nov, Z, (double)scale, 0);
    nm::hip_check(hipGetLastError(), "t2 target");
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int cc_guess_t2(cc_ctx* c, nm_mlp* net, const float* mu, const float* sd, float scale) {
  ABI_GUARD(c);
  int ni = 0, no = 0;
  if (!net || mlp_dims(net, &ni, nullptr, &no) != CC_OK || ni != 8 || no != 1 || !(scale > 0.0f))
    return CC_ERR_ARG;
  try {
    nm::ArenaScope sc(c->eng->arena());
    const int64_t tot = (int64_t)c->o * c->o * c->v * c->v, nov = (int64_t)c->o * c->v;
    float* F = (float*)c->eng->arena().alloc(tot * 4);
    float* Z = (float*)c->eng->arena().alloc((tot + 1) / 2);
    const int rc = cc_t2_features(c, mu, sd, F);
    if (rc != CC_OK) return rc;
    if (mlp_forward(net, tot, F, Z) != CC_OK) {
      c->err = std::string("network evaluation failed: ") + mlp_last_error(net);
      return CC_ERR_HIP;
    }
    nm::kc(nm::fill(c->s, c->t, 0.0, nov), "fill");
    const int g = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(nm::t2_map_kernel, dim3(g), dim3(256), 0, c->s, c->Gov.p, c->eps.p, c->o, c->v,
                       c->t + nov, Z, (double)scale, 1);
    nm::hip_check(hipGetLastError(), "t2 guess");
    // the network sees (i, a) and (j, b) in order: restore t_ij^ab = t_ji^ba
    nm::kc(nm::apply_metric(c->s, c->t, c->t, c->o, c->v, 2), "symmetrise");
    c->have_guess = true;
    nm::sync(*c);
    return CC_OK;
  } catch (const Error& e) {
    return fail(c, e);
  }
}

int nm_contract(const char* spec, double alpha, const double* A, const int64_t* dA, const double* B,
                const int64_t* dB, double beta, double* C, const int64_t* dC, int precision,
                void* stream) {
  if (!spec || !A || !B || !C || !dA || !dB || !dC) return CC_ERR_ARG;
  try {
    std::string s(spec);
    const size_t c1 = s.find(','), ar = s.find("->");
    if (c1 == std::string::npos || ar == std::string::npos || ar < c1) return CC_ERR_ARG;
    const std::string la = s.substr(0, c1), lb = s.substr(c1 + 1, ar - c1 - 1), lc = s.substr(ar + 2);
    if (la.size() > 6 || lb.size() > 6 || lc.size() > 6) return CC_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    static thread_local std::unique_ptr<nm::Engine> eng;
    if (!eng || eng->stream() != st) eng.reset(new nm::Engine(st));
    if (precision != CC_FP64 && precision != CC_FP32_REFINE && precision != CC_BF16X3_REFINE)
      return CC_ERR_ARG;
    eng->set_lowp(precision != CC_FP64);
    eng->set_bf16(precision == CC_BF16X3_REFINE);
    eng->set_lowp_min_flops(0.0);   // the test surface applies the mode to any size
    std::vector<int64_t> sa(dA, dA + la.size()), sb(dB, dB + lb.size()), sc(dC, dC + lc.size());
    nm::ArenaScope scope(eng->arena());
    nm::Graph G(*eng);
    const int ia = G.leaf(nm::tview(const_cast<double*>(A), sa));
    const int ib = G.leaf(nm::tview(const_cast<double*>(B), sb));
    const int ic = G.leaf(nm::tview(C, sc));
    nm::DView vc = nm::full_view(G.val(ic), lc);
    if (beta != 1.0) {
      int64_t n = 1;
      for (auto x : sc) n *= x;
      nm::kc(nm::axpby(st, C, C, 0.0, beta, n), "scale");
    }
    // views with repeated labels handled by the graph's view builder
    nm::Term t = nm::mul(alpha, nm::op(ia, la), nm::op(ib, lb), lc);
    const int out = G.node(sc, {t});
    int64_t n = 1;
    for (auto x : sc) n *= x;
    nm::kc(nm::axpby(st, C, G.val(out).p, 1.0, 1.0, n), "accumulate");
    (void)vc;
    nm::hip_check(hipStreamSynchronize(st), "sync");
    return CC_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

int cc_stats(const cc_ctx* c, double* out, int n) {
  if (!c || !out || n < 1) return CC_ERR_ARG;
  const double v[7] = {(double)c->n_residual, (double)c->n_right, (double)c->n_left,
                       (double)c->eng->gemm_flops(), (double)c->eng->arena().peak_bytes(),
                       (double)c->eng->arena().reserved_bytes(),
                       (double)c->eng->lowp_flops()};
  for (int k = 0; k < n && k < 7; ++k) out[k] = v[k];
  return CC_OK;
}

int nm_gemm(int precision, int ta, int tb, int M, int N, int K, double alpha, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta, double* C, int64_t ldc,
            void* stream) {
  return nm_gemm_tiled(precision, -1, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
}

int nm_gemm_tiled(int precision, int tile, int ta, int tb, int M, int N, int K, double alpha,
                  const void* A, int64_t lda, const void* B, int64_t ldb, double beta, double* C,
                  int64_t ldc, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 1) return CC_ERR_ARG;
  if (tile < -1 || tile >= nm::kBf16Tiles || (tile >= 0 && precision != CC_BF16X3_REFINE))
    return CC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (precision == CC_FP64)
    rc = nm::gemm_f64(st, ta != 0, tb != 0, M, N, K, 1, alpha, (const double*)A, lda, 0,
                      (const double*)B, ldb, 0, beta, C, ldc, 0);
  else if (precision == CC_FP32_REFINE)
    rc = nm::gemm_f32acc(st, ta != 0, tb != 0, M, N, K, 1, alpha, (const float*)A, lda, 0,
                         (const float*)B, ldb, 0, beta, C, ldc, 0);
  else if (precision == CC_BF16X3_REFINE) {
    // interleaved bfloat16 pairs: A [M][lda], B^T [N][ldb], lda, ldb >= 2 K
    if (ta || !tb || K % 32 || lda < 2 * (int64_t)K || ldb < 2 * (int64_t)K) return CC_ERR_ARG;
    rc = nm::gemm_bf16x3(st, M, N, K, 1, alpha, (const uint16_t*)A, lda, 0, (const uint16_t*)B, ldb, 0, beta,
                         C, ldc, 0, 0, tile);
    if (rc == -1) return CC_ERR_ARG;
  } else
    return CC_ERR_ARG;
  return rc == 0 ? CC_OK : CC_ERR_HIP;
}

int nm_eig_host(int m, const double* G, double* wr, double* wi, double* V) {
  if (m < 1 || !G || !wr || !wi || !V) return CC_ERR_ARG;
  std::vector<double> g(G, G + (size_t)m * m);
  std::vector<std::complex<double>> w, Vc;
  if (!nm::eig_nonsym(g, m, w, Vc)) return CC_ERR_NUMERIC;
  for (int k = 0; k < m; ++k) {
    wr[k] = w[k].real();
    wi[k] = w[k].imag();
    int imax = 0;
    for (int i = 1; i < m; ++i)
      if (std::abs(Vc[(size_t)k * m + i]) > std::abs(Vc[(size_t)k * m + imax])) imax = i;
    const std::complex<double> ph = std::conj(Vc[(size_t)k * m + imax]) / std::abs(Vc[(size_t)k * m + imax]);
    for (int i = 0; i < m; ++i) V[(size_t)k * m + i] = (Vc[(size_t)k * m + i] * ph).real();
  }
  return CC_OK;
}

}  // extern "C"
