// Internal kernel launchers of the tdmrg library (gfx950).  Not part of the
// public ABI.  All complex arrays are planar: an imaginary-plane offset
// (in elements) locates the imaginary part of every operand.
#pragma once
#include <hip/hip_runtime.h>

namespace tdmrg {

// Operand of a complex GEMM.  Element (row, col) of the stored matrix of
// batch b and reduction slice r sits at p + b*sb + r*sr + row*ld + col.
// For A the logical operand is (m, k): trans=0 stores A as [m][k], trans=1
// stores it as [k][m].  For B the logical operand is (k, n): trans=0 stores
// [k][n], trans=1 stores [n][k].  conj=1 conjugates the operand.
struct GemmOperand {
  const double* p;
  long im;
  long sb, sr, ld;
  int trans, conj;
  long sk = 0;  // pointer step per split-K chunk (see GemmArgs::ktot)
  int f32 = 0;  // stored as FP32 (p points to floats; offsets count floats); FP32 / BF16 arithmetic only
};

// C[b] = alpha * sum_{r < nred} opA(A[b,r]) opB(B[b,r]) + beta * C[b]
// Row i of C[b] starts at i * ldc, or, when c_mi > 0, at
// (i / c_mi) * c_so + (i % c_mi) * ldc (rows split into an outer and an
// inner index, for outputs written straight into a permuted layout).
struct GemmArgs {
  int M, N, K, nbatch, nred;
  int role;  // 0 generic; 1 / 2: first / last stage of H_eff,2 (own kernel names)
  GemmOperand A, B;
  double* C;
  long c_im, c_sb, ldc;
  double alpha_re, alpha_im, beta_re, beta_im;
  int c_mi = 0;
  long c_so = 0;
  // Split K: when ktot > 0 the launch has a third grid dimension of chunks;
  // chunk c covers the K indices [c K, min((c+1) K, ktot)) of every batch,
  // with operand pointers advanced by c * sk and C by c * c_sk.
  int ktot = 0;
  long c_sk = 0;
  // Channel mix inside the A loader (role 3, A not transposed, no split K):
  // A(m, k; r) = sum_e v_e X[w_e][m / mx_dout][sp_e][k] over the entries e of
  // CSR row r * mx_dout + m % mx_dout (col = w * mx_din + sp, values planar
  // [2][mx_nnz]), in entry order; X = A.p (imaginary plane at A.im) with
  // X[w][p][sp][k] at w * mx_ws + (p * mx_din + sp) * A.ld + k.
  const int* mx_rowptr = nullptr;
  const int* mx_col = nullptr;
  const double* mx_v = nullptr;
  long mx_nnz = 0, mx_ws = 0;
  int mx_din = 0, mx_dout = 0;
  // C stored as FP32 (FP32 / BF16 arithmetic only; no split K)
  int c_f32 = 0;
};

// F64: FP64 MFMA (3M complex products); F32: operands rounded to FP32,
// FP32 MFMA; BF16X3 / BF16X6: operands split into two / three bfloat16
// pieces, 3 / 6 piece products per real product on the BF16 MFMA, FP32
// accumulation.
enum class Arith { F64 = 0, F32 = 1, BF16X3 = 2, BF16X6 = 3 };

hipError_t launch_cgemm(const GemmArgs& g, Arith arith, hipStream_t s);
// Tile variant 0 = 64x64 (launch_cgemm, which takes 32x32 tiles for products
// of fewer than 64 such tiles), 1 = 128x64, 2 = 64x128 (K slices of 16), 3 =
// 64x64 with K slices of 32, 4 = 64x64 with K slices of 16 and two LDS
// stages, 5 = 64x64 with eight waves and K slices of 32; all agree bitwise.
constexpr int kGemmTileVariants = 6;
hipError_t launch_cgemm_tile(const GemmArgs& g, Arith arith, int variant, hipStream_t s);
// C[b] = alpha * sum_{s < S} P[s][b] + beta * C[b], summed in the order
// s = 0, 1, ...  P: planar [2][S][nbatch][M][N] (imaginary plane at
// S*nbatch*M*N); C[b] at b * c_sb, rows at ldc, stored as FP32 when c_f32.
hipError_t launch_splitk_reduce(const double* P, int S, int nbatch, int M, int N, double* C, long c_im,
                                long c_sb, long ldc, double alpha_re, double alpha_im, double beta_re,
                                double beta_im, int c_f32, hipStream_t s);
// Number of 64x64 output tiles of g (all batches).
int cgemm_tiles(const GemmArgs& g);
// Persistent grouped launch over np independent GEMMs (args and the prefix
// sums of their tile counts in device memory); all share the operand
// layouts trans_a / trans_b.
hipError_t launch_cgemm_grouped(const GemmArgs* args_dev, const int* tile_start_dev, int np, int trans_a,
                                int trans_b, int total_tiles, Arith arith, hipStream_t s);

// Sparse channel mixing (the MPO stages of the contractions):
//   out[c][p][s][q] = sum_{(w,s') in row (c,s)} v * in[w][p][s'][q]
// CSR over output rows c*dout+s; col[e] = w*din + s'.
// Row blocks of a channel operator for the multi-row channel kernel: the
// kMixRows consecutive output rows [B kMixRows, (B+1) kMixRows) share the
// distinct input columns bcol[bptr[B] .. bptr[B+1]) (ascending, each w *
// din + s'); bval [2][ncols][kMixRows] holds every row's coefficient of the
// column (zero where the row has no entry), bmask[u] the rows with a stored
// entry.  Each row still sums its entries in ascending column order, the
// order of its CSR row.
constexpr int kMixRows = 8;
struct MixBlocks {
  const int* bptr = nullptr;
  const int* bcol = nullptr;
  const double* bval = nullptr;
  const unsigned* bmask = nullptr;
  long ncols = 0;
};

struct MixArgs {
  const double* in;
  long in_im;
  double* out;
  long out_im;
  int P, Q, din, dout, nout;
  const int* rowptr;
  const int* col;
  const double* vre;
  const double* vim;
  MixBlocks blk;  // optional row blocks of the same operator (multi-row kernel)
  int f32 = 0;    // in and out stored as FP32 (in, out point to floats; offsets count floats)
};
hipError_t launch_mix(const MixArgs& a, hipStream_t s);
// np independent mixing stages in one launch; elem_start (device) holds the
// prefix sums of their output element counts (nout*dout*P*Q).
hipError_t launch_mix_grouped(const MixArgs* args_dev, const long* elem_start_dev, int np, long total,
                              hipStream_t s);

// ---- Lanczos / vector kernels (FP64, planar vectors of n complex) ----
// partial[j*nchunk + b] (complex, planar in two arrays) = sum over chunk b of
// conj(V_j[i]) * w[i], j < nv, V_j = V + j*vstride.
int dot_chunks(long n);
hipError_t launch_multidot(const double* V, long vstride, int nv, long n, const double* w,
                           double* part_re, double* part_im, hipStream_t s);
// out[j] (complex) = sum_b partial[j*nchunk + b], fixed order.  mode 0: write
// (re, im) to out_re/out_im[j]; mode 1 (norm): out_re[j] = sqrt(re).
hipError_t launch_reduce_partials(const double* part_re, const double* part_im, int nv, int nchunk,
                                  double* out_re, double* out_im, int mode, hipStream_t s);
// w[i] -= sum_j (cr[j] + i ci[j]) V_j[i]
hipError_t launch_multiaxpy(const double* V, long vstride, int nv, long n, const double* cr,
                            const double* ci, double* w, hipStream_t s);
// As launch_multiaxpy, and nrm[0] = ||w|| of the updated w (partials of the
// multidot chunking in part, fixed-order reduction).
hipError_t launch_multiaxpy_norm(const double* V, long vstride, int nv, long n, const double* cr,
                                 const double* ci, double* w, double* part, double* nrm, hipStream_t s);
// dst[0] = src[0] on the stream (device scalars)
hipError_t launch_copy_scalar(const double* src, double* dst, hipStream_t s);

// Forms of the Lanczos step kernels driven by a device counter jd = j (the
// step index), so that one step's launches are the same for every j and can
// be replayed as a graph: vector counts are j + 1 (grids sized for nv_max),
// scalars go to index j.
// (blocks do nothing while j + 1 < nv_min)
hipError_t launch_multidot_dev(const double* V, long vstride, const int* jd, int nv_max, long n, const double* w,
                               double* part_re, double* part_im, int nv_min, hipStream_t s);
hipError_t launch_reduce_partials_dev(const double* part_re, const double* part_im, const int* jd, int nv_max,
                                      int nchunk, double* out_re, double* out_im, int mode, hipStream_t s);
hipError_t launch_multiaxpy_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                                const double* ci, double* w, int nv_min, hipStream_t s);
// w -= sum_{k<=j} c_k v_k and the multidot partials of <v_k, w> for the
// updated w in one read of the basis, while j + 1 <= kGsFusedMax (does
// nothing beyond); bitwise equal to launch_multiaxpy_dev + launch_multidot_dev.
constexpr int kGsFusedMax = 8;
hipError_t launch_gs_fused_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                               const double* ci, double* w, double* part_re, double* part_im, hipStream_t s);
// beta[j] = ||w|| of the updated w
hipError_t launch_multiaxpy_norm_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                                     const double* ci, double* w, double* part, double* beta, hipStream_t s);
// dst[j] = src[j]
hipError_t launch_copy_scalar_dev(const double* src, double* dst, const int* jd, hipStream_t s);
// exp(-i tau T_{j+1}) e1 and the error estimate
hipError_t launch_tridiag_expm_dev(const double* alpha, const double* beta, const int* jd, double tau,
                                   double* c_re, double* c_im, double* err, hipStream_t s);
// x = w / beta[j], also stored as V[j + 1] when j + 1 < m_max
hipError_t launch_lanczos_next(const double* w, long n, const double* beta, double* V, long vstride, double* x,
                               const int* jd, int m_max, hipStream_t s);
// c = value / c += value (one device int)
hipError_t launch_counter_set(int* c, int value, hipStream_t s);
hipError_t launch_counter_add(int* c, int value, hipStream_t s);
// out[i] = scale * sum_j (cr[j] + i ci[j]) V_j[i]; scale read from *scale_dev.
hipError_t launch_combine(const double* V, long vstride, int nv, long n, const double* cr,
                          const double* ci, const double* scale_dev, double* out, hipStream_t s);
// dst = src / (*nrm) (zero when *nrm == 0)
hipError_t launch_scale_by_inv(const double* src, long n, const double* nrm, double* dst,
                               hipStream_t s);
// Lanczos bookkeeping after the first dot of step j: alpha[j] = Re(dot);
// coefficients for w -= alpha v_j + beta_{j-1} v_{j-1}.
hipError_t launch_lanczos_alpha(const double* dot_re, int j, double* alpha, const double* beta,
                                double* cr, double* ci, hipStream_t s);
// c = exp(-i tau T) e1 for T = tridiag(alpha[0..m-1], beta[0..m-2]); err =
// beta[m-1] * |c[m-1]|.  m <= 64.
hipError_t launch_tridiag_expm(const double* alpha, const double* beta, int m, double tau,
                               double* c_re, double* c_im, double* err, hipStream_t s);

// ---- SVD helpers ----
// interleave planar [2][n] into complex (re, im) pairs
hipError_t launch_interleave(const double* planar, long n, double* z, hipStream_t s);
// rank selection on descending S[nsv] (see tdmrg_svd_truncate); writes
// out_k[0] and out_disc[0]
hipError_t launch_choose_rank(const double* S, int nsv, double eps, int D_max, int sv_mode,
                              double tie_rel, int* out_k, double* out_disc, hipStream_t s);
// Singular values from the ascending eigenvalues lam[n] of a Gram matrix:
// S[j] = sqrt(max(lam[n-1-j], 0)), descending.
hipError_t launch_eig_to_sv(const double* lam, int n, double* S, hipStream_t s);
// Top-k eigenvectors of a Hermitian matrix stored column-major interleaved
// in Z (n x n, ascending order) as planar out:
//   transpose=0: out[i][j] = conj?(z_{n-1-j}[i])  ([2][n][k])
//   transpose=1: out[j][i] = conj?(z_{n-1-j}[i])  ([2][k][n])
// optionally divided by S[j] (rows or columns j; zero when S[j] == 0).
hipError_t launch_eigvec_extract(const double* Z, int n, int k, int conj, int transpose,
                                 double* out, hipStream_t s);
// One-sided (Hestenes) Jacobi SVD in one workgroup for small problems.
// left=1: the vectors are the conjugated rows of theta (nv = rows, length
// cols), so theta = Vacc W^H; left=0: the vectors are the columns of theta
// (nv = cols, length rows), so theta = W Vacc^H.  Wk [2][nv][len] and Vacc
// [2][nv][nv] (stored transposed: row j holds column j) are workspace; on
// exit sig[j] (descending) are the singular
// values and perm[j] the vector index holding the j-th one.
constexpr int kJacobiMaxVectors = 512;
hipError_t launch_jacobi_svd(const double* theta, int rows, int cols, int left, double* Wk,
                             double* Vacc, double* sig, int* perm, int max_sweeps, hipStream_t s);
// Outputs after rank selection (k kept):
//  mode 0: out1 = U [rows][k], out2 = Vh [k][cols] (divided by sig, zero rows
//          for sig == 0); mode 1: out1 = U, out2 = S Vh; mode 2: out1 = U S,
//  out2 = Vh.  left selects how Wk/Vacc were produced.  With left=1 the
//  factor Vh is W^H (divided by sig in mode 0); with left=0 the factor U is W
//  (U S in mode 2, divided by sig otherwise) and out2 = Vh = Vacc^H.
hipError_t launch_jacobi_assemble(const double* Wk, const double* Vacc, const double* sig,
                                  const int* perm, int rows, int cols, int left, int k, int mode,
                                  double* out1, double* out2, hipStream_t s);
// Scale row j (by_rows=1) or column j of a planar [2][rows][cols] matrix by
// f(S[j]): S[j] (inv=0) or 1/S[j] (inv=1, zero when S[j] == 0).
hipError_t launch_scale_sv(double* m, int rows, int cols, const double* S, int by_rows, int inv,
                           hipStream_t s);

hipError_t launch_fill(double* p, long n, double v, hipStream_t s);
// out[b][i][j] = conj(in[b][j][i]) for nb planar n x n matrices (plane size nb*n*n)
hipError_t launch_conj_transpose(const double* in, int nb, int n, double* out, hipStream_t s);
// x *= (re + i im), planar vector of n complex
hipError_t launch_cscale(double* x, long n, double re, double im, hipStream_t s);

// ---- adjoints ----
// Z[j][i] /= (s_keep[i]^2 - s_perp[j]^2) (planar kp x k; zero for pairs closer
// than 1e-14 s_all[0]^2)
hipError_t launch_gap_scale(double* Z, int kp, int k, const double* s_perp, const double* s_keep, const double* s_all,
                            hipStream_t s);
// X[i][j] /= S[j]^2 (zero when S[j] == 0), planar rows x cols
hipError_t launch_scale_cols_inv2(double* X, int rows, int cols, const double* S, hipStream_t s);
// out = in^H for a planar rows x cols matrix
hipError_t launch_conj_transpose_rect(const double* in, int rows, int cols, double* out, hipStream_t s);

// ---- Hermitian eigensolver (n <= kHeevMax) ----
constexpr int kHeevMax = 512;
// Largest order the SVD routes hand to it: the reduction streams the trailing
// block through one CU (about 50 GB/s measured), so beyond about 240 rocSOLVER
// zheevd is faster (n = 192: 2.1 ms reduction + 0.8 ms dstedc + 0.2 ms
// back-transformation against 4.5 ms; n = 384: 13.7 ms against 9.8 ms).
constexpr int kHeevRoute = 240;
// Householder reduction of the Hermitian n x n C (planar row-major, lower
// triangle read) to the real tridiagonal (d[n], e[n-1]) = Q^H C Q in one
// workgroup; reflectors v_j in the rows of V [2][n][n] (v_j[0] = 1), tau
// [2][n]; A [2][n][n] is scratch.
hipError_t launch_hetrd(const double* C, int n, double* A, double* V, double* d, double* e, double* tau,
                        hipStream_t s);
// Q z_{n-1-j} for j < k (the k largest eigenpairs, largest first) from the
// column-major real eigenvectors Z of the tridiagonal matrix (ascending):
// transpose=0: out[i][j] ([2][n][k]), transpose=1: out[j][i] ([2][k][n]),
// conj=1 conjugates.
hipError_t launch_unmtr(const double* V, const double* tau, const double* Z, int n, int k, int transpose, int conj,
                        double* out, hipStream_t s);

// ---- subspace-iteration SVD ----
constexpr int kMaxSubspace = 512;  // largest block of the subspace iteration
// x[t] = uniform in [-1, 1) from a counter-based generator, t < n
hipError_t launch_randfill(double* x, long n, unsigned long long seed, hipStream_t s);
// the same for columns j0 .. b-1 of a planar row-major p x b matrix
hipError_t launch_randfill_cols(double* x, int p, int b, int j0, unsigned long long seed, hipStream_t s);
// Blocked Cholesky factorisation with triangular inverse (the recursion and
// its GEMMs run on the host side).  gram_colscale: d_i = 1/sqrt(G_ii) and
// G <- diag(d) G diag(d) + shift * 1 (planar b x b; status[0] = 1 on a zero
// or non-finite diagonal).  chol_leaf: for an n x n block A (upper triangle,
// planar with imaginary plane at im_a, row stride lda), A = R^H R and Rinv =
// R^(-1) written as a full n x n block (zeros below the diagonal); status[0]
// = 2 when A is not positive definite.  rowscale: T[i][j] *= d[i].  Status
// words are only written on failure.  b <= kMaxSubspace, n <= kCholLeaf.
constexpr int kCholLeaf = 64;
hipError_t launch_gram_colscale(double* G, int b, double* d, int* status, hipStream_t s, double shift = 0.0);
hipError_t launch_chol_leaf(const double* A, long im_a, long lda, int n, double* Rinv, long im_r, long ldr,
                            int* status, hipStream_t s);
hipError_t launch_rowscale(double* T, int b, const double* d, hipStream_t s);
// out[j] = 2-norm of column j < ncols of a planar row-major matrix (imaginary
// plane at offset im, row stride ld); part holds colnorm_part_doubles(ncols).
hipError_t launch_colnorms(const double* P, long im, int rows, long ld, int ncols, double* part, double* out,
                           hipStream_t s);
long colnorm_part_doubles(int ncols);
// Rank selection (as launch_choose_rank) from the leading nb singular values
// and the Frobenius norm norm[0] of the whole matrix.
hipError_t launch_choose_rank_partial(const double* S, int nb, const double* norm, double eps, int D_max,
                                      int sv_mode, double tie_rel, int* out_k, double* out_disc, hipStream_t s);


// Damped one-sided transform of sampled C(t) (planar [2][N], t_k = k dt):
// sigma[m] = (1/(pi hbar)) Re sum_k w_k C_k exp(i E_m t_k/hbar - t_k/tau),
// trapezoid weights.
hipError_t launch_spectrum(const double* C, int N, double dt, double tau, double hbar, const double* E, int M,
                           double* sigma, hipStream_t s);

// Whole-MPS building blocks.  mpo_apply: one site of the MPO x MPS product,
// out[(a wl + w)][s][(b wr + y)] = sum_t W[w][y][s][t] A[a][t][b] (planar;
// W [2][wl][wr][d][d]).  block_copy: dst[a0 + a][s][b0 + b] = c src[a][s][b]
// (dst [2][Ld][d][Rd], src [2][Ls][d][Rs]; hipErrorInvalidValue when the
// block does not fit).
hipError_t launch_mpo_apply(const double* W, int wl, int wr, int d, const double* A, int Dl, int Dr, double* out,
                            hipStream_t s);
hipError_t launch_block_copy(double* dst, int Ld, int Rd, const double* src, int Ls, int Rs, int d, int a0, int b0,
                             double cr, double ci, hipStream_t s);

// out[j][i][e] = in[i][j][e] (+ out[j][i][e] when acc) for i < n1, j < n2,
// e < q; planar complex, imaginary planes at in + in_im and out + out_im.
// in and out must not overlap.
hipError_t launch_swap_outer(const double* in, long in_im, int n1, int n2, long q, double* out, long out_im,
                             bool acc, hipStream_t s);

// out[i][j] = A[i ld + j] from interleaved complex A into planar out
// [2][nrow][ncol]; mask 1 keeps j >= i, 2 keeps j <= i, 0 everything.
hipError_t launch_extract_ld(const double* A, long ld, int nrow, int ncol, int mask, double* out, hipStream_t s);
}  // namespace tdmrg
