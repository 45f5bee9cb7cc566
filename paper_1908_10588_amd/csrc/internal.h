// Internal state of the tdmrg library: handles behind the opaque ABI types,
// the device workspace and the host-side drivers of the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <array>
#include <atomic>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tdmrg.h"
#include "kernels.h"

namespace tdmrg {

// Two-site channel operator W12[wl][wr][(s,t)][(s',t')] = sum_wc W1[wl][wc][s][s'] W2[wc][wr][t][t']
// as a device CSR over output rows (wr, s*d2+t); entries (wl*(d1 d2) + s'*d2 + t').
// Device row blocks of a channel operator (see MixBlocks).
struct DevBlocks {
  int* bptr = nullptr;
  int* bcol = nullptr;
  double* bval = nullptr;
  unsigned* bmask = nullptr;
  long ncols = 0;
  MixBlocks view() const {
    MixBlocks b;
    b.bptr = bptr;
    b.bcol = bcol;
    b.bval = bval;
    b.bmask = bmask;
    b.ncols = ncols;
    return b;
  }
};

struct PairOp {
  int* rowptr = nullptr;
  int* col = nullptr;
  double* v = nullptr;  // [2][nnz]
  long nnz = 0;
  DevBlocks blk;
};

// Row blocks of a CSR operator (rows in groups of kMixRows) on the host.
struct HostBlocks {
  std::vector<int> bptr, bcol;
  std::vector<double> bval;  // [2][ncols][kMixRows]
  std::vector<unsigned> bmask;
};
void build_mix_blocks(int nrows, const int* rowptr, const int* col, const double* vre, const double* vim,
                      HostBlocks* out);
// Bytes of the row blocks of an operator with nnz stored entries (upper bound).
size_t mix_blocks_bytes(long nrows, long nnz);

// A growable device allocation owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A caller-owned device buffer the context draws its workspace from
// (tdmrg_ctx_create with an arena): first fit over a free list of
// 256-byte-aligned blocks, merged with their neighbours when released.
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> size
  std::map<size_t, size_t> used_blocks;  // offset -> size
};

// Optional per-stage timing of the H_eff,2 product with HIP events on the
// context stream: stage 0 = L * theta GEMM, 1 = W_i mixing, 2 = W_{i+1}
// mixing, 3 = (.) R^T GEMM.  Events are read back after the stream has been
// synchronised (flush).
struct Profiler {
  bool on = false;
  struct Pending {
    hipEvent_t a, b;
    int stage;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[4] = {0, 0, 0, 0};
  double flops[4] = {0, 0, 0, 0};
  double bytes[4] = {0, 0, 0, 0};
  long launches[4] = {0, 0, 0, 0};
};

}  // namespace tdmrg

struct tdmrg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  std::string err;
  // workspace
  tdmrg::DevBuf xa, xb;          // contraction intermediates
  tdmrg::DevBuf kry, wvec;       // Krylov basis, Lanczos work vector
  tdmrg::DevBuf theta;           // two-site tensor of the sweep
  tdmrg::DevBuf svd_z, svd_u, svd_vt, svd_s, svd_e;  // rocSOLVER operands
  tdmrg::DevBuf envA, envB;      // observables
  tdmrg::DevBuf small;           // Lanczos scalars, partial sums, flags
  tdmrg::DevBuf meta;            // per-problem descriptors of grouped launches
  tdmrg::DevBuf batch;           // intermediates and Krylov vectors of a batch wave
  tdmrg::DevBuf bscal, bpart;    // per-problem Lanczos scalars, partial sums
  tdmrg::DevBuf vjpA, vjpB, vjpC, vjpD, vjpL, vjpR, vjpU, vjpV;  // adjoint workspace
  tdmrg::DevBuf sub;             // subspace-iteration SVD blocks
  tdmrg::DevBuf adjw, adjt;      // truncation adjoint: full SVD and transposed operands
  tdmrg::DevBuf kryU, wvecU, smallU;  // second Krylov basis of the exponential's adjoint
  tdmrg::DevBuf splitk;          // partial products of split-K GEMMs
  tdmrg::DevBuf cqr;             // Cholesky QR of a divided SVD factor (small Jacobi route)
  tdmrg::DevBuf qr;              // first-pass factor and status words of qr_split
  tdmrg::DevBuf gbuf, gsmall;    // scratch of the global integrators
  tdmrg::DevBuf hqr;             // Householder factorisation of qr_householder
  tdmrg::DevBuf heev;            // Hermitian eigensolver: reduction, reflectors, tridiagonal eigenvectors
  tdmrg::Arena arena;            // caller-owned workspace (base == nullptr: the library allocates)
  tdmrg::DevBuf rocws;           // rocBLAS/rocSOLVER workspace drawn from the arena
  int svd_schedule = 0;          // first Rayleigh-Ritz check: 0 adaptive, 1 at iteration 1
  int mpo_apply = 0;             // global steps: 0 direct MPO x MPS product + compression, 1 variational fit
  int svd_first_check = 3;       // iteration at which the last subspace SVD converged
  std::map<int, tdmrg_wop*> ident_ops;  // identity channel maps for one-site adjoints
  size_t batch_budget = 0;       // bytes per batch wave (0 = 60% of free memory)
  double* host = nullptr;        // pinned host scratch for read-backs
  tdmrg::Profiler prof;
  // fused two-site channel operators, keyed by (W1 id, W2 id)
  std::map<std::pair<long, long>, tdmrg::PairOp> pairs;
  int fuse_mode = 1;             // 0 never fuse the channel stages, 1 cost model, 2 always
  int mix_in_gemm = 0;           // fused channel stage inside the last GEMM's A loader
  int svd_method = 0;            // 0 automatic, 1 Jacobi, 2 Gram + eigensolver, 3 subspace iteration
  int eig_method = 0;            // Hermitian eigensolver: 0 library reduction (n <= kHeevRoute), 1 rocSOLVER zheevd
  int chan_gemm = 1;             // channel stages as GEMMs: 0 never, 1 cost model, 2 always
  int autotune = 1;              // GEMM tile autotuning (tdmrg_ctx_set_autotune)
  int verbose = 0;               // progress lines on stderr (tdmrg_ctx_set_verbose)
  std::map<std::array<int, 8>, int> tiles;  // tuned tile variant per shape class
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  // Lanczos step graphs (tdmrg_ctx_set_graphs): one captured step per operand
  // set, replayed for every step j (the kernels read j from a device counter).
  // Valid while the global graph epoch is unchanged: every reallocation of a
  // workspace buffer and every destruction of an operator or MPS advances it.
  int graphs = 1;
  hipStream_t cap_stream = nullptr;  // capture stream (the context's stream may be the null stream)
  struct StepGraph {
    hipGraphExec_t exec = nullptr;  // nullptr: the step could not be captured
    unsigned long epoch = 0;        // graph epoch at capture
  };
  std::map<std::vector<long>, StepGraph> lgraphs;
  unsigned long lgraph_epoch = 0;  // epoch of the last sweep of stale entries
  long graph_counts[3] = {0, 0, 0};  // captures, replayed steps, eager steps
  long quad_nodes_used = 0, quad_calls = 0;  // quadrature nodes / calls of the exponential adjoints
  long long svd_count[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // see tdmrg_ctx_svd_counters
};

struct tdmrg_wop {
  tdmrg_ctx* ctx = nullptr;
  long id = 0;  // unique per created operator (cache key)
  int wl = 0, wr = 0, d = 0;
  std::vector<double> host;  // planar [2][wl][wr][d][d]
  // forward CSR: rows (c < wr, s), entries (w < wl, s')  value W[w][c][s][s']
  // backward CSR: rows (c < wl, s), entries (w < wr, s') value W[c][w][s][s']
  int* f_rowptr = nullptr; int* f_col = nullptr; double* f_v = nullptr; int f_nnz = 0;
  int* b_rowptr = nullptr; int* b_col = nullptr; double* b_v = nullptr; int b_nnz = 0;
  tdmrg::DevBlocks f_blk;  // row blocks of the forward CSR (multi-row channel kernel)
  tdmrg_wop* adj = nullptr;  // adjoint operator, created on demand
  // dense matrix forms for the channel stages as GEMMs, created on demand:
  // left  [2][d*wr][wl*d]: row s*wr + c, column w*d + s' holds W[w][c][s][s']
  // right [2][wr*d][wl*d]: row c*d + s, column w*d + s' holds W[w][c][s][s']
  double* dense_l = nullptr;
  double* dense_r = nullptr;
};

struct tdmrg_mpo {
  tdmrg_ctx* ctx = nullptr;
  int n = 0, n_el = 0;
  std::vector<int> pop_site;      // chain site whose operator gives population i
  std::vector<int> dims, wdims;
  std::vector<tdmrg_wop*> W;
  std::vector<tdmrg_wop*> ident;  // w = 1 identity on every site
  std::vector<tdmrg_wop*> proj;   // w = 1 |i><i| on the electronic site (per-state: n_i)
  std::vector<double*> dense;     // device copies of W[s], planar [2][wl][wr][d][d] (MPO x MPS)
};

struct tdmrg_mps {
  tdmrg_ctx* ctx = nullptr;
  int n = 0;
  std::vector<int> dims, bond, cap;
  std::vector<double*> site;  // device [2][Dl][d][Dr] at capacity
  // environments of the MPO they were built for
  const tdmrg_mpo* env_mpo = nullptr;
  bool env_valid = false;
  std::vector<double*> L, R;
};

namespace tdmrg {

// Advanced whenever device memory that a captured graph may reference is
// freed or moved (see tdmrg_ctx::lgraphs).
void graph_epoch_bump();
unsigned long graph_epoch();
// Destroys the context's cached graphs.
void graphs_clear(tdmrg_ctx* ctx);

tdmrg_status validate_model(const tdmrg_ctx* ctx, const tdmrg_model* m);
// MPO of the model as dense host arrays [2][wl][wr][d][d].  keep_zero keeps
// terms whose coupling is zero as channels (with zero weight), so that the
// channel structure does not depend on which couplings vanish (the gradient
// with respect to a zero coupling needs its channel).
tdmrg_status build_mpo_host(const tdmrg_ctx* ctx, const tdmrg_model* m, std::vector<int>* dims,
                            std::vector<int>* wdims, std::vector<std::vector<double>>* W,
                            std::vector<int>* pop_sites, bool keep_zero = false);
// tdmrg_mpo_build with the keep_zero choice above.
tdmrg_status mpo_build(tdmrg_ctx* ctx, const tdmrg_model* model, bool keep_zero, tdmrg_mpo** out);

tdmrg_status fail(const tdmrg_ctx* ctx, tdmrg_status st, const std::string& msg);
// Device memory of the context's workspace: from the caller's arena when the
// context has one (ENOMEM when no free block fits), else hipMalloc.
tdmrg_status dev_alloc(tdmrg_ctx* ctx, size_t bytes, void** out);
void dev_free(tdmrg_ctx* ctx, void* p);

// ---- workspace plan of a 2TDVP sweep (workspace.cpp) ----
// Upper bounds, in bytes, of every workspace buffer a tdmrg_tdvp2_sweep (and
// tdmrg_observables) on an MPS with bond capacities caps may need, over every
// route the steps can take (fused or separate channel stages, the three SVD
// routes and the fallback, split K).
struct WsPlan {
  size_t theta = 0, small = 0, kry = 0, wvec = 0, xa = 0, xb = 0, splitk = 0;
  size_t svd_u = 0, svd_z = 0, svd_s = 0, svd_e = 0, svd_vt = 0, sub = 0, cqr = 0, heev = 0;
  size_t envA = 0, envB = 0, pairs = 0, rocws = 0;
  size_t total() const;  // every buffer rounded up to the arena's alignment
};
// W: host MPO site tensors [2][wl][wr][d][d]; fuse_mode as tdmrg_ctx::fuse_mode.
WsPlan plan_sweep(const std::vector<int>& dims, const std::vector<int>& wdims, const std::vector<int>& caps,
                  int krylov_max, const std::vector<std::vector<double>>& W, int fuse_mode);
// Arena contexts: every buffer of the plan for (mps, mpo, krylov_max)
// reserved before the sweep launches anything (ENOMEM, nothing modified, when
// the arena is too small); no-op for contexts without an arena.
tdmrg_status reserve_sweep(tdmrg_ctx* ctx, const tdmrg_mps* mps, const tdmrg_mpo* mpo, int krylov_max);
// Arena contexts: rocBLAS/rocSOLVER get at least `bytes` of the arena as
// their workspace (rocblas_set_workspace).  No-op without an arena.
tdmrg_status rocws_reserve(tdmrg_ctx* ctx, size_t bytes);
// Bytes of rocSOLVER workspace the library allows for a Hermitian
// eigenproblem or Householder factorisation of order n (an upper bound of
// what rocSOLVER asks for on gfx950).
size_t rocsolver_ws_bound(long n);
// bytes of ctx->heev for the hand-written Hermitian eigensolver of order n
size_t heev_bytes(int n);
// Hand-written Hermitian eigensolver, n <= kHeevMax, in two phases over
// ctx->heev: heev_values reduces C (planar row-major n x n, lower triangle
// read) to tridiagonal form and solves the tridiagonal problem (rocSOLVER
// dstedc): lam[n] ascending, *info (device) nonzero when it did not converge;
// heev_vectors then writes the eigenvectors of the k largest eigenvalues,
// largest first, in the layout of launch_unmtr (transpose, conj).
tdmrg_status heev_values(tdmrg_ctx* ctx, const double* C, int n, double* lam, int* info);
tdmrg_status heev_vectors(tdmrg_ctx* ctx, int n, int k, int transpose, int conj, double* out);
// The same for the Householder factorisations (LQ/QR and Q) of order n.
size_t rocsolver_qr_ws_bound(long n);
// Whether the fused channel operator of (W1, W2) pays by the cost model
// (fuse_mode 1; 2 always, 0 never), and the number of its entries before
// cancellation (an upper bound of its nonzeros).  W1 [2][wl][wc][d1][d1],
// W2 [2][wc][wr][d2][d2] host planar.
bool pair_fusion_plan(const double* W1, int wl, int wc, int d1, const double* W2, int wr, int d2, int fuse_mode,
                      long* products);
// GEMM launch with split K for few-tile long reductions and the tile-variant
// autotuner (both keep results deterministic).
hipError_t tuned_cgemm(tdmrg_ctx* ctx, const GemmArgs& g, Arith ar, hipStream_t s);
tdmrg_status ensure(tdmrg_ctx* ctx, DevBuf& b, size_t bytes);
// Operator from a host planar [2][wl][wr][d][d] array (device CSR in both
// channel directions).
tdmrg_status wop_make(tdmrg_ctx* ctx, int wl, int wr, int d, const double* planar, tdmrg_wop** out);
// Adjoint (per-block conjugate transpose, channels unchanged) of W, created
// on first use and owned by W.
tdmrg_status wop_adjoint(tdmrg_ctx* ctx, const tdmrg_wop* W, const tdmrg_wop** out);
// Dense matrix form of W for the left (right = 0) or right (right = 1) site
// of a pair (see tdmrg_wop), built on first use.
tdmrg_status wop_dense(tdmrg_ctx* ctx, const tdmrg_wop* W, int right, const double** out);
tdmrg_status heff2_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                       const tdmrg_wop* W2, const double* R, const double* theta, const double* ybar,
                       double* Lbar, double* W1bar, double* W2bar, double* Rbar, double* thetabar,
                       bool accumulate);
// thetabar is overwritten; the operand cotangents accumulate when acc.
tdmrg_status local_expm2_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                             const tdmrg_wop* W2, const double* R, const double* theta_in, double tau,
                             const double* ybar, double* Lbar, double* W1bar, double* W2bar, double* Rbar,
                             double* thetabar, int nquad, double tol, int m_max, bool acc);
// Adjoints of the other steps of a time step (adjoint.cpp).  Mbar of the
// one-site exponential is overwritten; every other cotangent accumulates.
// Environments of mps for mpo (allocated at capacity; rebuilt when not valid):
// L[0] = R[n] = 1, R[b] from the sites right of bond b.
tdmrg_status ensure_envs(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo);
tdmrg_status ident_wop(tdmrg_ctx* ctx, int w, const tdmrg_wop** out);
tdmrg_status local_expm1_vjp(tdmrg_ctx* ctx, int Dl, int Dr, const double* L, const tdmrg_wop* W,
                             const double* R, const double* M_in, double tau, const double* ybar, double* Lbar,
                             double* Wbar, double* Rbar, double* Mbar, int nquad, double tol, int m_max);
tdmrg_status env_left_vjp(tdmrg_ctx* ctx, const double* Lin, const tdmrg_wop* W, const double* bra, int Db,
                          int Db2, const double* ket, int Dk, int Dk2, const double* Obar, double* Lin_bar,
                          double* Wbar, double* bra_bar, double* ket_bar);
tdmrg_status env_right_vjp(tdmrg_ctx* ctx, const double* Rin, const tdmrg_wop* W, const double* bra, int Db,
                           int Db2, const double* ket, int Dk, int Dk2, const double* Obar, double* Rin_bar,
                           double* Wbar, double* bra_bar, double* ket_bar);
tdmrg_status theta_form_vjp(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr, const double* M,
                            const double* B, const double* thetabar, double* Mbar, double* Bbar);
// Adjoint of svd_truncate's mode 1 (out1 = U, out2 = S Vh) or mode 2 (out1 =
// U S, out2 = Vh) at kept rank k for a loss invariant under the gauge of the
// kept bond; thetabar is overwritten.
tdmrg_status svd_trunc_vjp(tdmrg_ctx* ctx, int m, int n, const double* theta, int mode, const double* out1,
                           const double* out2, const double* S, int k, const double* out1_bar, const double* out2_bar,
                           double* thetabar);
// The cached fused channel operator of (W1, W2), built on first use; null
// when fusion is not worthwhile by the cost model (or disabled).
tdmrg_status pair_op(tdmrg_ctx* ctx, const tdmrg_wop* W1, const tdmrg_wop* W2, const PairOp** out);
// Whether the channel stages of H_eff,2 for this shape run as dense GEMMs
// (tdmrg_ctx_set_channel_gemm; cost model in mode 1).
bool channel_gemm_pays(const tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const tdmrg_wop* W1,
                       const tdmrg_wop* W2);
void pair_release(tdmrg_ctx* ctx);
// Accumulate the elapsed times of recorded events (stream must be idle).
// Event pair around one profiled launch (stage 0..3), its algorithmic flops and bytes.
tdmrg_status prof_begin(tdmrg_ctx* ctx, Profiler::Pending* p, int stage);
tdmrg_status prof_end(tdmrg_ctx* ctx, Profiler::Pending& p, double flops, double bytes);
tdmrg_status prof_flush(tdmrg_ctx* ctx);
void prof_release(tdmrg_ctx* ctx);

// y = H_eff,2 theta; all planar device pointers.
tdmrg_status heff2(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                   const tdmrg_wop* W2, const double* R, const double* theta, double* y, Arith ar);
tdmrg_status heff1(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* L, const tdmrg_wop* W,
                   const double* R, const double* M, double* y, Arith ar);
// out = alpha (L W1 W2 R) theta + beta out with environments between
// different bra and ket bases (FP64, separate channel stages):
//   out[a][s][t][b] = sum L[w][a][a'] W1[w][x][s][s'] W2[x][y][t][t'] R[y][b][b'] theta[a'][s'][t'][b'],
// L [2][wl][Dlo][Dli], R [2][wr][Dro][Dri], theta [2][Dli][d1][d2][Dri],
// out [2][Dlo][d1][d2][Dro] (the pair update of a variational MPS fit).
tdmrg_status heff2_rect(tdmrg_ctx* ctx, int Dlo, int Dli, int d1, int d2, int Dro, int Dri, const double* L,
                        const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, const double* theta, double* out,
                        double alpha_re, double alpha_im, double beta);
// y = H_eff,0 C for a Dl x Dr bond matrix; L [w][Dl][Dl], R [w][Dr][Dr].
tdmrg_status heff0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R, const double* C,
                   double* y, Arith ar);
// Lout[w'][a][a'] from Lin[w][b][b'], bra [Db][d][Db2], ket [Dk][d][Dk2]
tdmrg_status env_left(tdmrg_ctx* ctx, const double* Lin, const tdmrg_wop* W, const double* bra,
                      int Db, int Db2, const double* ket, int Dk, int Dk2, double* Lout, Arith ar);
// Rout[w][a][a'] from Rin[w'][b][b'], bra [Db][d][Db2], ket [Dk][d][Dk2]
tdmrg_status env_right(tdmrg_ctx* ctx, const double* Rin, const tdmrg_wop* W, const double* bra,
                       int Db, int Db2, const double* ket, int Dk, int Dk2, double* Rout, Arith ar);
tdmrg_status theta_form(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr, const double* M,
                        const double* B, double* theta);
struct ExpmResult {
  int iters = 0;
  bool converged = true;
};
tdmrg_status local_expm(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, bool two_site, const double* L,
                        const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, double* theta,
                        double tau, double tol, int m_max, Arith ar, ExpmResult* res);
// sites = 2, 1 or 0 (zero-site: shape {Dl, 1, 1, Dr, w, 1, w}, no operators)
tdmrg_status local_expm_sites(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, int sites, const double* L,
                              const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R, double* theta,
                              double tau, double tol, int m_max, Arith ar, ExpmResult* res);
// C = exp(-i tau H_eff,0) C in place
tdmrg_status local_expm0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R, double* C,
                         double tau, double tol, int m_max, Arith ar, ExpmResult* res);
// M = Q C (right = false: M rows x cols with rows >= cols, Q^H Q = 1, C
// cols x cols) or M = C Q (right = true: rows <= cols, Q Q^H = 1, C rows x
// rows); Q must not alias M.  *cholesky_ok = false when the Cholesky QR
// passes broke down and the SVD route produced the split.
tdmrg_status qr_split(tdmrg_ctx* ctx, int rows, int cols, const double* M, bool right, double* Q, double* C,
                      bool* cholesky_ok);
// The same split by Householder QR (rocSOLVER) for any shape and rank, with
// k = min(rows, cols): left M = Q C (Q rows x k, C k x cols), right M = C Q
// (C rows x k, Q k x cols).
tdmrg_status qr_householder(tdmrg_ctx* ctx, int rows, int cols, const double* M, bool right, double* Q, double* C);
// A Lanczos basis kept for evaluating exp(-i t H) x at several times t.
struct KrylovBasis {
  double* V = nullptr;  // m planar vectors of n complex (stride 2n)
  long n = 0;
  int m = 0;
  double *alpha = nullptr, *beta = nullptr, *beta0 = nullptr, *c_re = nullptr, *c_im = nullptr, *err = nullptr;
};
// Builds the basis of (H_eff,2, x) to the tolerance of exp(-i tau H) x
// (two-site shape; storage in the given buffers); the basis then serves
// every time t with |t| <= |tau| of the same sign.
tdmrg_status expm_basis(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                        const tdmrg_wop* W2, const double* R, const double* x, double tau, double tol, int m_max,
                        DevBuf& Vbuf, DevBuf& wbuf, DevBuf& sbuf, KrylovBasis* kb);
// out = |x| V exp(-i t T) e1 from a basis.
tdmrg_status expm_from_basis(tdmrg_ctx* ctx, const KrylovBasis& kb, double t, double* out);
tdmrg_status heff2_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes, const double* const* L,
                           const tdmrg_wop* const* W1, const tdmrg_wop* const* W2, const double* const* R,
                           const double* const* theta, double* const* y, Arith ar);
tdmrg_status local_expm_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                const double* const* L, const tdmrg_wop* const* W1,
                                const tdmrg_wop* const* W2, const double* const* R, double* const* theta,
                                double tau, double tol, int m_max, Arith ar, int* iters, int* nonconv);
// mode 0: out1 = U, out2 = Vh, S_out = S;  1: out1 = U, out2 = S Vh;
// 2: out1 = U S, out2 = Vh.  Outputs are packed at the kept rank k.
tdmrg_status svd_truncate(tdmrg_ctx* ctx, int rows, int cols, const double* theta, double eps,
                          int D_max, int sv_mode, double tie_rel, int k_cap, int mode, double* out1,
                          double* out2, double* S_out, int* k, double* disc);

// ---- the no-allocation form of H_eff,2 theta (noalloc.hip) ----
// Looks up the device address of the library's fixed scratch array on
// `device` (current) once; called when a context is created.
hipError_t noalloc_init(int device);
size_t noalloc_scratch_bytes();
// Doubles of scratch heff2_noalloc needs for a shape.
double noalloc_heff2_doubles(const tdmrg_heff_shape& s);
// y = H_eff,2 theta with the intermediates in the scratch array (ESHAPE when
// they do not fit); no allocation, no autotuning, no split K.
tdmrg_status heff2_noalloc(tdmrg_ctx* ctx, const tdmrg_heff_shape& s, const double* L, const tdmrg_wop* W1,
                           const tdmrg_wop* W2, const double* R, const double* theta, double* y, Arith ar);

}  // namespace tdmrg
