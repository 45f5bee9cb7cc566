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
};

// C[b] = alpha * sum_{r < nred} opA(A[b,r]) opB(B[b,r]) + beta * C[b]
struct GemmArgs {
  int M, N, K, nbatch, nred;
  int role;  // 0 generic; 1 / 2: first / last stage of H_eff,2 (own kernel names)
  GemmOperand A, B;
  double* C;
  long c_im, c_sb, ldc;
  double alpha_re, alpha_im, beta_re, beta_im;
};

enum class Arith { F64 = 0, F32 = 1 };

hipError_t launch_cgemm(const GemmArgs& g, Arith arith, hipStream_t s);

// Sparse channel mixing (the MPO stages of the contractions):
//   out[c][p][s][q] = sum_{(w,s') in row (c,s)} v * in[w][p][s'][q]
// CSR over output rows c*dout+s; col[e] = w*din + s'.
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
};
hipError_t launch_mix(const MixArgs& a, hipStream_t s);

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
// U[r][j] = VT[j + r*ldv] (complex interleaved), planar out [2][rows][k];
// optionally times S[j].
hipError_t launch_unpack_left(const double* VT, int ldv, int rows, int k, const double* S,
                              int scale, double* out, hipStream_t s);
// Vh[j][c] = U2[c + j*ldu], planar out [2][k][cols]; optionally times S[j].
hipError_t launch_unpack_right(const double* U2, int ldu, int cols, int k, const double* S,
                               int scale, double* out, hipStream_t s);

hipError_t launch_fill(double* p, long n, double v, hipStream_t s);

}  // namespace tdmrg
