/*
 * tdmrg.h -- C ABI of the MI355X (gfx950) two-site TDVP library.
 *
 * The library evolves a matrix product state (MPS) under an el-vib (vibronic)
 * Hamiltonian with the two-site time-dependent variational principle
 * (2TDVP) of Xie et al., "Time-dependent density matrix renormalization group
 * quantum dynamics for realistic chemical systems", arXiv 1908.10588,
 * Section 2.1.2 (eq. two-site Hamiltonian and the procedure after it).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: energies in eV, times in fs, hbar = TDMRG_HBAR_EV_FS eV*fs.
 *  - Complex tensors are stored *planar*: the whole real plane followed by the
 *    whole imaginary plane, each row-major with the last index fastest.
 *    "[2][a][b][c]" below means re[a][b][c] then im[a][b][c], FP64.
 *  - Index order of the tensors (bra/output index first):
 *      MPS site tensor   A[alpha_{i-1}][sigma_i][alpha_i]          (eq. MPS tensor)
 *      MPO site tensor   W[w_{i-1}][w_i][sigma][sigma']            (eq. MPO)
 *      left environment  L[w][a][a']    a = bra (output), a' = ket (input)
 *      right environment R[w][b][b']    b = bra (output), b' = ket (input)
 *      two-site tensor   theta[a][s][t][b]
 *  - Pointers documented as "device" must point to device memory of the
 *    context's GPU (for example torch tensors on that device); they are
 *    borrowed for the duration of the call.  "host" pointers are read (or
 *    written) during the call only.
 *  - All device work is ordered on the context's HIP stream.  Entry points
 *    that return scalars to the host (ranks, iteration counts, observables)
 *    synchronise that stream.
 *  - Every function returns a tdmrg_status.  Arguments are validated before
 *    any launch; on TDMRG_EINVAL/TDMRG_ESHAPE nothing is modified.
 *    tdmrg_last_error() returns a message describing the last failure.
 *  - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef TDMRG_H
#define TDMRG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDMRG_HBAR_EV_FS 0.6582119569

typedef enum {
  TDMRG_OK = 0,
  TDMRG_EINVAL = 1,       /* invalid argument (NaN, negative size, bad order ...) */
  TDMRG_ENOMEM = 2,       /* device or host allocation failed */
  TDMRG_EDEVICE = 3,      /* HIP / rocSOLVER error, no usable GPU */
  TDMRG_ENOCONV = 4,      /* Lanczos did not reach its tolerance in m_max steps (result written) */
  TDMRG_ESHAPE = 5,       /* shapes inconsistent with each other or with a handle */
  TDMRG_EUNSUPPORTED = 6  /* valid request this build does not implement */
} tdmrg_status;

/* Arithmetic of the tensor contractions (H_eff * theta and environments).
 * Lanczos vectors, orthogonalisation, the tridiagonal exponential and the
 * SVD always run in FP64. */
typedef enum {
  TDMRG_FP64 = 0,   /* FP64 MFMA, FP64 accumulation */
  TDMRG_FP32 = 1,   /* operands rounded to FP32, FP32 MFMA, FP32 accumulation */
  TDMRG_BF16X3 = 2, /* BF16-split products: each operand rounded to FP32 and split into two
                       bfloat16 pieces (16 significant bits), three piece products per real
                       product (after Henry, Tang and Heinecke, ARITH 2019) on the BF16 MFMA,
                       FP32 accumulation: about 2^-16 relative error per product */
  TDMRG_BF16X6 = 3  /* three bfloat16 pieces (24 bits), six piece products per real product
                       (every product of order <= 2), FP32 accumulation: the FP32 level */
} tdmrg_precision;

typedef struct tdmrg_ctx tdmrg_ctx;
typedef struct tdmrg_wop tdmrg_wop; /* one MPO site tensor resident on the device */
typedef struct tdmrg_mpo tdmrg_mpo;
typedef struct tdmrg_mps tdmrg_mps;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` whose work is ordered on
 * `hip_stream` (a hipStream_t; NULL = the default stream).
 * Workspace (the contraction intermediates of eq. two-site Hamiltonian, the
 * Krylov basis of the local exponentials, the SVD blocks of the DBSS
 * truncation, the environment chains of the observables, the fused channel
 * operators, and rocBLAS/rocSOLVER's own workspace):
 *  - arena == NULL, arena_bytes == 0: the library allocates it on the device
 *    and grows it on demand;
 *  - otherwise `arena` is a caller-owned device buffer of this GPU (for
 *    example a torch.empty tensor) of arena_bytes bytes, which must outlive
 *    the context.  Every workspace buffer is carved from it (first fit,
 *    256-byte blocks) and nothing else is allocated for workspace; a sweep
 *    reserves its whole plan (tdmrg_workspace_query) before it launches
 *    anything and returns TDMRG_ENOMEM, with nothing modified, when the
 *    arena is too small; other calls return TDMRG_ENOMEM when a buffer they
 *    need does not fit.  Site tensors, environments and operators (the MPS
 *    and MPO handles) are allocated by their own create calls.
 * EINVAL if only one of arena / arena_bytes is given or the arena is not
 * device memory of `device`; EDEVICE if no such device exists. */
tdmrg_status tdmrg_ctx_create(int device, void* hip_stream, void* arena, size_t arena_bytes, tdmrg_ctx** out);
void tdmrg_ctx_destroy(tdmrg_ctx* ctx);
/* Message of the last failure on `ctx` (or of the last failed create when
 * ctx is NULL).  Valid until the next call on the context. */
const char* tdmrg_last_error(const tdmrg_ctx* ctx);
tdmrg_status tdmrg_ctx_synchronize(tdmrg_ctx* ctx);
/* Bytes of device workspace currently held by the context. */
tdmrg_status tdmrg_ctx_workspace_bytes(const tdmrg_ctx* ctx, size_t* bytes);

/* Per-stage timing of every H_eff,2 product (eq. two-site Hamiltonian) made
 * on the context, measured with HIP events on its stream.  Stage 0: the
 * L*theta GEMM, 1: the W_i channel stage, 2: the W_{i+1} channel stage, 3: the
 * R GEMM.  flops are algorithmic (8 per complex multiply-add; channel stages
 * count the stored nonzeros of W), bytes the compulsory operand traffic of
 * the stage.  Enabling (on != 0) or disabling resets the counters;
 * get_profile synchronises the stream. */
typedef struct {
  double ms[4];
  double flops[4];
  double bytes[4];
  long launches[4];
} tdmrg_profile;
tdmrg_status tdmrg_ctx_set_profiling(tdmrg_ctx* ctx, int on);
tdmrg_status tdmrg_ctx_get_profile(tdmrg_ctx* ctx, tdmrg_profile* out);

/* -------------------------------------------------------------------- model */

/* Vibronic coupling constants of the el-vib Hamiltonian, Section 2.2
 * (eqs. Hel_2, Hvib_2, Helvib_2):
 *   H = sum_i E_i |i><i| + sum_{i!=j} V_ij |i><j| + sum_I omega_I (n_I + 1/2)
 *     + sum_{I,i,j} g1[I][i][j] q_I |i><j|
 *     + sum_k g2[k] * Q_k * (|i_k><j_k| + h.c. if i_k != j_k),
 *       Q_k = q_I q_J (I != J) or q_I^2 (I == J, exact truncated elements).
 * q = (b^+ + b)/sqrt(2) in the basis |0>..|nbasis-1>.  One electronic site of
 * dimension n_el, or one site per state (el_per_state).  All arrays are host
 * memory, copied during the call. */
typedef struct {
  int n_el, n_modes;
  const double* E;       /* [n_el] */
  const double* V;       /* [n_el*n_el], symmetric; the diagonal is ignored */
  const double* omega;   /* [n_modes] hbar*omega_I (eV) */
  const int* nbasis;     /* [n_modes] local dimension d_I >= 2 */
  const double* g1;      /* [n_modes*n_el*n_el], symmetric in the last two indices */
  int n_g2;
  const int *g2_I, *g2_J, *g2_i, *g2_j; /* [n_g2] mode and state indices */
  const double* g2;      /* [n_g2] coefficients */
  const int* order;      /* chain order: [n_modes+1] with -1 = the electronic site, or, when
                            el_per_state = 1, [n_modes+n_el] with -1-i = the site of state i */
  int el_per_state;      /* 0: one electronic site of dimension n_el; 1: one site of dimension
                            2 (empty, occupied) per state, as in the paper's ordering study:
                            |i><i| -> n_i, |i><j| + h.c. -> a_i^+ a_j + a_j^+ a_i (hard-core
                            occupation operators; the dynamics stays in the one-excitation
                            sector, so no exchange sign arises) */
} tdmrg_model;

/* MPO of the model Hamiltonian (eq. MPO) by a finite-state construction.
 * Channels on a bond: "nothing applied", "term complete", one channel per
 * electronic operator (or operator product) pending completion.  Terms whose
 * first operator lies left of the electronic site share channels by their
 * remaining operators, the others by their applied operators.
 * EINVAL: NaN/inf constants, nbasis < 2, order not a permutation, index out
 * of range. */
tdmrg_status tdmrg_mpo_build(tdmrg_ctx* ctx, const tdmrg_model* model, tdmrg_mpo** out);
void tdmrg_mpo_destroy(tdmrg_mpo* mpo);
/* n_sites; dims[n_sites] local dimensions; wdims[n_sites+1] MPO bond
 * dimensions (either array may be NULL). */
tdmrg_status tdmrg_mpo_info(const tdmrg_mpo* mpo, int* n_sites, int* dims, int* wdims);
/* Host copy of W[site] as [2][w_l][w_r][d][d]. */
tdmrg_status tdmrg_mpo_get_site(const tdmrg_mpo* mpo, int site, double* planar_host);
/* The device operator of one site (owned by the MPO). */
const tdmrg_wop* tdmrg_mpo_site(const tdmrg_mpo* mpo, int site);

/* Bytes of workspace arena (tdmrg_ctx_create) that tdmrg_tdvp2_sweep and
 * tdmrg_observables need for this model on an MPS created with D_cap = D_max
 * (every bond capped at min(D_max, its full-rank bound)), with at most
 * krylov_max Lanczos vectors per local exponential: an upper bound over every
 * route the steps can take (separate or fused channel stages, the Jacobi,
 * Gram and subspace SVD routes and the fallback, split K).  For the
 * benchmark's 24-mode model at D_max 128 and 40 Krylov vectors it is about
 * 18 GB: the Krylov basis (40 two-site tensors of up to 1.5e7 complex, 9.4
 * GB) and the two contraction intermediates (15 channels each, 3.5 GB).  Host only (no device needed); the precision does not change
 * the size.  EINVAL for an invalid model, D_max < 1, krylov_max outside
 * 1..64. */
tdmrg_status tdmrg_workspace_query(const tdmrg_model* model, int D_max, int krylov_max, tdmrg_precision precision,
                                   size_t* bytes);

/* Host-only form of the same construction (no device, no context): the
 * number of sites, dims[n] and wdims[n+1] (either may be NULL), and, when
 * planar_host != NULL, W[site] as [2][w_l][w_r][d][d].  Same validation as
 * tdmrg_mpo_build. */
tdmrg_status tdmrg_mpo_host_query(const tdmrg_model* model, int* n_sites, int* dims, int* wdims);
tdmrg_status tdmrg_mpo_host_site(const tdmrg_model* model, int site, double* planar_host);

/* An MPO site tensor W[w_l][w_r][d][d] (host, planar) uploaded to the device
 * together with its channel-block sparsity (zero d x d blocks and zero
 * entries are skipped by the contraction kernels). */
tdmrg_status tdmrg_wop_create(tdmrg_ctx* ctx, int wl, int wr, int d, const double* planar_host,
                              tdmrg_wop** out);
void tdmrg_wop_destroy(tdmrg_wop* w);
/* Number of stored nonzero entries of the operator. */
tdmrg_status tdmrg_wop_nnz(const tdmrg_wop* w, long* nnz);

/* ---------------------------------------------------------------------- MPS */

/* Product state |occ_0> x ... x |occ_{n-1}> (bond dimensions 1, right-canonical
 * with the orthogonality centre on site 0; Section 3.1 starts from such a
 * state).  D_cap bounds every bond dimension the state will ever hold; device
 * storage for every site is reserved at that capacity. */
tdmrg_status tdmrg_mps_init(tdmrg_ctx* ctx, const tdmrg_mpo* mpo, const int* occ, int D_cap,
                            tdmrg_mps** out);
tdmrg_status tdmrg_mps_copy(const tdmrg_mps* src, tdmrg_mps** out);
void tdmrg_mps_destroy(tdmrg_mps* mps);
/* bonds[n_sites+1] current bond dimensions. */
tdmrg_status tdmrg_mps_bond_dims(const tdmrg_mps* mps, int* bonds);
/* Replace site `site` by the host tensor [2][Dl][d][Dr].  The caller keeps the
 * state consistent (matching neighbouring bonds, right-canonical sites 1..n-1
 * before tdvp2_sweep).  ESHAPE when Dl/Dr exceed the capacity. */
tdmrg_status tdmrg_mps_set_site(tdmrg_mps* mps, int site, int Dl, int Dr, const double* planar_host);
/* Dimensions of a site and, when planar_host != NULL, a host copy [2][Dl][d][Dr]. */
tdmrg_status tdmrg_mps_get_site(const tdmrg_mps* mps, int site, int* Dl, int* d, int* Dr,
                                double* planar_host);

/* ------------------------------------------- single steps (device operands) */

typedef struct { int Dl, d1, d2, Dr, wl, wc, wr; } tdmrg_heff_shape;

/* y = H_eff,2 theta (eq. two-site Hamiltonian):
 *   y[a][s][t][b] = sum L[w][a][a'] W1[w][x][s][s'] W2[x][y][t][t'] R[y][b][b'] theta[a'][s'][t'][b'].
 * L [2][wl][Dl][Dl], R [2][wr][Dr][Dr], theta and y [2][Dl][d1][d2][Dr]: device.
 * W1 (wl x wc, d1) and W2 (wc x wr, d2) must match the shape (ESHAPE).
 * y must not alias any input. */
tdmrg_status tdmrg_heff2_apply(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                               const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                               const double* theta, double* y, tdmrg_precision prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product
 * of tdmrg_heff2_apply, same operands, layouts and kernels (the channel
 * stages always run as the two sparse passes; no tile autotuning, no split
 * K), with its two intermediates, 16 * (max(wl, wr) + wc) * Dl*d1*d2*Dr
 * bytes, in a fixed 64 MiB device array that the library holds on every GPU
 * it is loaded on until the process ends.  Nothing is allocated or freed
 * (no hipMalloc, hipFree or allocating library routine).  ESHAPE when the
 * intermediates exceed 64 MiB.  All calls on one GPU share the array, so
 * calls that may overlap on one GPU (other streams, other host threads)
 * race and must be ordered by the caller.  Results agree with
 * tdmrg_heff2_apply to rounding. */
tdmrg_status tdmrg_heff2_apply_noalloc(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                       const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                       const double* theta, double* y, tdmrg_precision prec);

/* y = H_eff,1 M (eq. one-site Hamiltonian 1); shape uses Dl, d1, Dr, wl, wr
 * (d2 and wc ignored).  M and y [2][Dl][d1][Dr]. */
tdmrg_status tdmrg_heff1_apply(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                               const tdmrg_wop* W, const double* R, const double* M, double* y,
                               tdmrg_precision prec);

/* theta <- exp(-i tau H_eff) theta by Lanczos with full (two-pass classical
 * Gram-Schmidt) re-orthogonalisation; tau = dt/hbar in 1/eV, signed (the
 * backward one-site step of eq. backward TDVP uses a negative tau).
 * two_site selects H_eff,2 (W2 used) or H_eff,1 (W2 ignored).  Stops when
 * beta_m |e_m^T exp(-i tau T_m) e_1| <= tol or after m_max (<= 64) steps;
 * *iters receives the number of H_eff applications.  ENOCONV: result
 * written, tolerance not met. */
tdmrg_status tdmrg_local_expm(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, int two_site,
                              const double* L, const tdmrg_wop* W1, const tdmrg_wop* W2,
                              const double* R, double* theta_inout, double tau, double tol,
                              int m_max, tdmrg_precision prec, int* iters);

/* y = H_eff,0 C (eq. zero-site Hamiltonian): the two environments of a bond
 * meet on the MPO bond between them,
 *   y[a][b] = sum_{w,a',b'} L[w][a][a'] C[a'][b'] R[w][b][b'].
 * L [2][w][Dl][Dl], R [2][w][Dr][Dr], C and y [2][Dl][Dr]: device; y must
 * not alias an input. */
tdmrg_status tdmrg_heff0_apply(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R,
                               const double* C, double* y, tdmrg_precision prec);

/* C <- exp(-i tau H_eff,0) C, the Lanczos exponential of tdmrg_local_expm
 * with the zero-site operator (the 1TDVP backward step uses tau < 0).
 * Same tolerance, iteration and status rules as tdmrg_local_expm. */
tdmrg_status tdmrg_local_expm0(tdmrg_ctx* ctx, int Dl, int Dr, int w, const double* L, const double* R,
                               double* C_inout, double tau, double tol, int m_max, tdmrg_precision prec,
                               int* iters);

/* Orthonormal split of a site tensor read as a rows x cols matrix (the
 * left-orthonormalisation M = L Q of the 1TDVP procedure in Section 2.1.2,
 * and its mirror image).  right = 0: M = Q C with Q rows x cols, Q^H Q = 1,
 * C cols x cols (needs cols <= rows); right = 1: M = C Q with Q rows x cols,
 * Q Q^H = 1, C rows x rows (needs rows <= cols); ESHAPE otherwise.  Two
 * column-scaled Cholesky QR passes and C as the exact projection of M on Q;
 * where a Cholesky pass breaks down (M numerically rank deficient), or the
 * bond exceeds 512 (the largest Cholesky block), the split is taken from
 * Householder QR (rocSOLVER), which holds for any rank, and *cholesky_ok
 * (optional) is 0.  Device buffers, planar; none may alias another.
 * Synchronises. */
tdmrg_status tdmrg_qr_split(tdmrg_ctx* ctx, int rows, int cols, const double* M, int right, double* Q,
                            double* C, int* cholesky_ok);

/* Batched / persistent form: n independent two-site problems of uneven
 * shapes (shapes[p], operands L[p], W1[p], W2[p], R[p], theta[p], y[p] as in
 * tdmrg_heff2_apply).  Each of the four stages of the product runs as ONE
 * persistent grouped launch over the tiles (GEMM stages) or output elements
 * (channel stages) of all problems; a fixed grid walks the global work list,
 * so every workgroup exits after a bounded number of items.  Problems are
 * processed in consecutive waves whose intermediates fit the batch budget
 * (tdmrg_ctx_set_batch_budget; default 60% of free device memory).
 * Host arrays of pointers, read during the call. */
tdmrg_status tdmrg_heff2_apply_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                       const double* const* L, const tdmrg_wop* const* W1,
                                       const tdmrg_wop* const* W2, const double* const* R,
                                       const double* const* theta, double* const* y,
                                       tdmrg_precision prec);
/* theta[p] <- exp(-i tau H_eff,2[p]) theta[p] for every problem, the Lanczos
 * steps of tdmrg_local_expm advanced in lockstep (one grouped H_eff product
 * per Krylov step over the problems still iterating).  iters[n] (nullable)
 * receives each problem's number of H_eff applications.  ENOCONV: results
 * written, some problem missed the tolerance. */
tdmrg_status tdmrg_local_expm_batched(tdmrg_ctx* ctx, int n, const tdmrg_heff_shape* shapes,
                                      const double* const* L, const tdmrg_wop* const* W1,
                                      const tdmrg_wop* const* W2, const double* const* R,
                                      double* const* theta_inout, double tau, double tol, int m_max,
                                      tdmrg_precision prec, int* iters);
/* The two MPO channel stages of H_eff,2 * theta can run as one pass through
 * the two-site channel operator sum_wc W_i[.][wc] (x) W_{i+1}[wc][.] (built on
 * the host on first use and cached per operator pair), which saves the
 * write and read of the middle intermediate.  mode 0: never, 1: when the
 * cost model favours it (default), 2: always.  Results agree to rounding. */
tdmrg_status tdmrg_ctx_set_fusion(tdmrg_ctx* ctx, int mode);
/* When the channel stages run fused (above), the fused pass can run inside
 * the A-operand loader of the last GEMM stage (each A tile is formed from
 * the first stage's output as it is loaded, in the same summation order),
 * which removes the channel kernel and the write and read of its output,
 * but serialises three dependent gathers (row pointer, column, value) per
 * entry in the loader: on the benchmark the last stage then takes 3.4 ms
 * against 1.2 + 0.7 ms for the GEMM and channel kernel.  on = 1 or 0 (a
 * separate channel kernel, default).  Results agree to rounding. */
tdmrg_status tdmrg_ctx_set_mix_in_gemm(tdmrg_ctx* ctx, int on);
/* The two MPO channel stages of H_eff,2 * theta as dense GEMMs on the MFMA
 * units (intermediates in the layouts [a][w_l][s'][t'][b'] and
 * [a][s][w_c][t'][b'], operators as dense (s, w_c) x (w_l, s') and
 * (w_r, t) x (w_c, t') matrices) instead of the sparse channel pass, which
 * pays off when the operators are dense.  mode 0: never, 1: when the cost
 * model favours it (default), 2: always.  Results agree to rounding; applies
 * to single and batched products. */
tdmrg_status tdmrg_ctx_set_channel_gemm(tdmrg_ctx* ctx, int mode);
/* Runtime GEMM tile autotuning (default on): the first call of each shape
 * class (operand transposes, precision, power-of-two buckets of M, N, K * nred
 * and the batch count) that overwrites its output and has at least 2e8
 * multiply-adds times every tile variant (0: 64x64 complex outputs per
 * workgroup, 1: 128x64, 2: 64x128, 3: 64x64 with K slices of 32, 4: 64x64
 * with two LDS stages, 5: 64x64 with eight waves and K slices of 32) with
 * events on the context stream (best of three runs after an untimed one)
 * and keeps the fastest.  The variants agree
 * bitwise, so results do not depend on it.
 * Tuning is skipped while profiling is on. */
tdmrg_status tdmrg_ctx_set_autotune(tdmrg_ctx* ctx, int on);
/* The tuned classes: *n = their number; when entries != NULL, up to cap rows
 * of 9 ints [trans_a, trans_b, precision, log2 M, log2 N, log2 (K nred),
 * log2 nbatch, channel mix in the A loader (0/1), variant] (bucket b holds
 * sizes in (2^(b-1), 2^b]). */
tdmrg_status tdmrg_ctx_tile_table(tdmrg_ctx* ctx, int cap, int* n, int* entries);
/* Lanczos step graphs (default on).  The kernels of one Lanczos step read
 * the step index from a device counter, so their launches are the same for
 * every step: they are captured once per operand set (problem shape,
 * operators, environments, workspace, tau) as a hipGraph and replayed for
 * every further step, also in later calls with the same operands (a sweep
 * over a saturated MPS reuses them every time step).  Results are bitwise
 * those of the eager launches.  Cached graphs are dropped whenever device
 * memory they reference may have moved (workspace growth, destruction of an
 * operator or MPS).  Off while profiling (tdmrg_ctx_set_profiling). */
tdmrg_status tdmrg_ctx_set_graphs(tdmrg_ctx* ctx, int on);
/* out[3] = {graphs captured, Lanczos steps replayed from graphs, steps
 * launched eagerly} since the context was created. */
tdmrg_status tdmrg_ctx_graph_counters(const tdmrg_ctx* ctx, long* out);
/* Progress lines on stderr from long calls (level 1: one line per time step
 * of tdmrg_tdvp2_population_grad's forward and reverse passes); 0 = quiet
 * (default).  EINVAL for a negative level. */
tdmrg_status tdmrg_ctx_set_verbose(tdmrg_ctx* ctx, int level);
/* Device-memory budget (bytes) of one batch wave; 0 restores the default. */
tdmrg_status tdmrg_ctx_set_batch_budget(tdmrg_ctx* ctx, size_t bytes);

/* ---------------------------------------------------------------- adjoints */
/* Cotangent convention: for a real loss f and complex z, zbar = df/dRe z +
 * i df/dIm z.  Outputs are overwritten; any output pointer may be NULL (not
 * computed).  FP64.  Device arrays: Lbar [2][wl][Dl][Dl], W1bar
 * [2][wl][wc][d1][d1] (dense, every entry of W_i), W2bar [2][wc][wr][d2][d2],
 * Rbar [2][wr][Dr][Dr], thetabar [2][Dl][d1][d2][Dr]. */

/* Vector-Jacobian product of y = H_eff,2 theta (eq. two-site Hamiltonian)
 * for f = Re<ybar, y>: thetabar = H_eff,2^H ybar; every operand cotangent is
 * the contraction of ybar with the conjugated product of the other operands
 * (environment-like contractions on the same kernels as the product). */
tdmrg_status tdmrg_heff2_apply_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                   const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                   const double* theta, const double* ybar, double* Lbar,
                                   double* W1bar, double* W2bar, double* Rbar, double* thetabar);
/* Vector-Jacobian product of y = exp(-i tau H_eff,2) theta_in (the local
 * forward step of the procedure after eq. two-site Hamiltonian):
 * thetabar = exp(+i tau H^H) ybar; operand cotangents from the Frechet
 * derivative of the exponential, int_0^1 of the H_eff VJP at
 * v_s = exp(-i tau s H) theta_in with cotangent i tau exp(+i tau (1-s) H^H) ybar,
 * by nquad-point Gauss-Legendre quadrature (exponentially accurate in
 * nquad for the analytic integrand).  tol / m_max as in tdmrg_local_expm. */
tdmrg_status tdmrg_local_expm_vjp(tdmrg_ctx* ctx, const tdmrg_heff_shape* shape, const double* L,
                                  const tdmrg_wop* W1, const tdmrg_wop* W2, const double* R,
                                  const double* theta_in, double tau, const double* ybar, double* Lbar,
                                  double* W1bar, double* W2bar, double* Rbar, double* thetabar, int nquad,
                                  double tol, int m_max);

/* theta[a][s][t][b] = sum_m M[a][s][m] B[m][t][b]  (the two-site tensor of
 * the procedure after eq. two-site Hamiltonian).  M [2][Dl][d1][Dm],
 * B [2][Dm][d2][Dr], theta [2][Dl][d1][d2][Dr]: device. */
tdmrg_status tdmrg_theta_form(tdmrg_ctx* ctx, int Dl, int d1, int Dm, int d2, int Dr,
                              const double* M, const double* B, double* theta);

/* SVD of theta reshaped to (Dl d1) x (d2 Dr) in FP64 and the DBSS truncation
 * (Section 2.1.1): k = the smallest rank whose relative discarded weight
 * sum_{j>=k} s_j^2 <= eps sum_j s_j^2 (sv_mode 0), or every s_j >= eps s_0
 * (sv_mode 1), or all min(rows, cols) values (sv_mode 2); then k <= D_max
 * and a multiplet s_k >= (1 - tie_rel) s_{k-1} > 0 at the cut is kept whole.
 * Writes U [2][Dl][d1][k], S [k] and Vh [2][k][d2][Dr] (device, capacity
 * k_cap >= k, else ESHAPE), the rank *k and the discarded weight *disc. */
tdmrg_status tdmrg_svd_truncate(tdmrg_ctx* ctx, int Dl, int d1, int d2, int Dr, const double* theta,
                                double eps, int D_max, int sv_mode, double tie_rel, int k_cap,
                                double* U, double* S, double* Vh, int* k, double* disc);
/* How truncated SVDs of the context are computed (the rank rule and the
 * outputs are the same for all):
 *   0 automatic (default): 1 for small problems (and for small ones that keep
 *     tiny singular values), 3 when 2 (D_max + oversampling) <= min(rows, cols),
 *     else 2;
 *   1 one-sided Jacobi on theta in one workgroup (at most 512 vectors on the
 *     orthonormal side, else EUNSUPPORTED);
 *   2 Gram matrix + full Hermitian eigensolver (see tdmrg_ctx_set_eigensolver);
 *   3 subspace iteration with Rayleigh-Ritz for the leading D_max + oversampling
 *     triplets (not for sv_mode 2: EUNSUPPORTED), continuing with 2 when it
 *     does not settle. */
tdmrg_status tdmrg_ctx_set_svd_method(tdmrg_ctx* ctx, int method);
/* The Hermitian eigensolver of the SVD's Gram route and of the Rayleigh-Ritz
 * step of the subspace iteration (the eigenpairs of an n x n Gram matrix or
 * Rayleigh quotient):
 *   0 (default) for n <= 240: Householder reduction to real tridiagonal form
 *     in one workgroup, rocSOLVER's divide and conquer dstedc on the
 *     tridiagonal matrix, back-transformation of the eigenvectors by the
 *     library's kernels; larger n as 1 (faster there);
 *   1 rocSOLVER zheevd.
 * Both are backward stable; the eigenvectors of clustered eigenvalues may
 * differ between them within the cluster.  EINVAL for other values. */
tdmrg_status tdmrg_ctx_set_eigensolver(tdmrg_ctx* ctx, int method);
/* Counters since context creation: out[0] Jacobi SVDs, [1] Gram + eigensolver
 * SVDs, [2] subspace SVDs, [3] their total iterations, [4] subspace runs that
 * did not settle, [5] subspace runs stopped by a failed factorisation
 * (both continue with the Gram route, counted in [1]), [6] Rayleigh-Ritz
 * checks (eigensolver calls) of the subspace runs, [7] one-site splits
 * (tdmrg_qr_split in the 1TDVP sweep) that took the SVD route. */
tdmrg_status tdmrg_ctx_svd_counters(tdmrg_ctx* ctx, long long out[8]);
/* When the subspace SVD runs its first Rayleigh-Ritz check (one Hermitian
 * eigensolver call per check): 0 (default) at the iteration at which the
 * previous subspace SVD of this context converged (at least 2, at most 8),
 * with the power steps before it orthonormalised by a shifted Cholesky QR
 * pass plus plain passes; 1 at the first iteration.  Both converge to the
 * same tolerance; 0 needs fewer eigensolver calls. */
tdmrg_status tdmrg_ctx_set_svd_schedule(tdmrg_ctx* ctx, int schedule);

/* Environment updates (projection of H onto the enlarged block basis):
 *  left : Lout[x][a][a'] = sum conj(A[b][s][a]) Lin[w][b][b'] W[w][x][s][s'] A[b'][s'][a']
 *         Lin [2][wl][Dl][Dl], A [2][Dl][d][Dr], Lout [2][wr][Dr][Dr];
 *  right: Rout[w][a][a'] = sum conj(B[a][s][b]) W[w][x][s][s'] Rin[x][b][b'] B[a'][s'][b']
 *         Rin [2][wr][Dr][Dr], B [2][Dl][d][Dr], Rout [2][wl][Dl][Dl]. */
tdmrg_status tdmrg_env_update_left(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* Lin,
                                   const tdmrg_wop* W, const double* A, double* Lout,
                                   tdmrg_precision prec);
tdmrg_status tdmrg_env_update_right(tdmrg_ctx* ctx, int Dl, int d, int Dr, const double* Rin,
                                    const tdmrg_wop* W, const double* B, double* Rout,
                                    tdmrg_precision prec);

/* ------------------------------------------------------------- time stepping */

typedef struct {
  int precision;      /* tdmrg_precision of the contractions */
  double krylov_tol;  /* default 1e-12 (relative to the norm of the vector) */
  int krylov_max;     /* default 40, at most 64 */
  int sv_mode;        /* 0 relative discarded weight (default), 1 s_j < eps s_0, 2 keep all */
  double tie_rel;     /* default 1e-12 */
} tdmrg_opts;

typedef struct {
  double max_disc, sum_disc; /* discarded weight of this step */
  int max_krylov;            /* most Lanczos steps of any local exponential */
  int total_krylov;          /* H_eff applications in this step */
  int not_converged;         /* local exponentials that hit krylov_max */
  double seconds[4];         /* host wall time: expm2, svd, env, expm1 */
} tdmrg_step_stats;

/* One symmetric 2TDVP time step of length dt_fs (procedure after eq.
 * two-site Hamiltonian, read as a left-to-right half-sweep with
 * exp(-i H dt/2hbar) on every pair and a right-to-left half-sweep back,
 * each pair except the last of a half-sweep followed by the one-site
 * backward step exp(+i H_eff,1 dt/2hbar) of eq. backward TDVP).  The MPS
 * must be right-canonical with its centre on site 0 (as left by mps_init
 * and by this function).  D_max <= the MPS capacity.  opts may be NULL
 * (defaults); stats may be NULL.  ENOCONV: step completed, some local
 * exponential missed its tolerance (counted in stats). */
tdmrg_status tdmrg_tdvp2_sweep(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs,
                               int D_max, double eps, const tdmrg_opts* opts,
                               tdmrg_step_stats* stats);

/* One symmetric 1TDVP time step of length dt_fs (the one-site procedure of
 * Section 2.1.2 with eqs. one-site TDSE and zero-site Hamiltonian, read as
 * the two-site step is): left to right, every site i is evolved with
 * exp(-i H_eff,1 dt/2hbar), split M_i = A_i C (tdmrg_qr_split), C evolved
 * backward with exp(+i H_eff,0 dt/2hbar) and absorbed into site i+1; then
 * the mirror image from right to left; no backward step after the last
 * site of a half-sweep.  Bond dimensions never change and nothing is
 * truncated, so norm and energy are conserved up to the Krylov tolerance;
 * every bond must fit the blocks on both of its sides (ESHAPE).  The MPS
 * must be right-canonical with its centre on site 0 and is left that way.
 * opts: precision, krylov_tol, krylov_max (sv_mode and tie_rel unused); may
 * be NULL.  stats (optional): seconds[] = forward one-site exponentials,
 * splits, environment updates, backward zero-site exponentials; discarded
 * weights are zero.  ENOCONV: step completed, some local exponential missed
 * its tolerance. */
tdmrg_status tdmrg_tdvp1_sweep(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs,
                               const tdmrg_opts* opts, tdmrg_step_stats* stats);

/* Spectrum from the autocorrelation (the pyrazine spectra of Section 3.1,
 * damping time tau): sigma[m] = (1/(pi hbar)) Re sum_k w_k C_k
 * exp(i E[m] t_k/hbar - t_k/tau), t_k = k dt_fs, k = 0 .. n_t-1, trapezoid
 * weights w_k (dt, halved at both ends); the one-sided transform, which
 * assumes C(-t) = conj(C(t)).  C [2][n_t] (planar C(t_k) = <psi(0)|psi(t_k)>,
 * as tdmrg_observables returns per step), E [n_E] in eV, sigma [n_E] in 1/eV:
 * device.  n_t >= 2, n_E >= 1, dt_fs, tau_fs > 0 (a huge tau means no
 * damping); EINVAL otherwise.  Stream-ordered. */
tdmrg_status tdmrg_spectrum(tdmrg_ctx* ctx, int n_t, double dt_fs, const double* C, double tau_fs, int n_E,
                            const double* E, double* sigma);

/* One time step of a global integrator on the whole MPS (Section 2.1.1):
 * method 0 = the global Krylov method (eqs. Krylov subspace, global Krylov):
 * Lanczos basis v_0 = psi/|psi|, v_{j+1} from H v_j - alpha_j v_j -
 * beta_{j-1} v_{j-1} with every H application and every sum compressed,
 * psi(t + dt) = |psi| sum_k c_k v_k, c = exp(-i dt/hbar T) e_1, stopping when
 * beta_j |c_j| <= tol or at m_max (<= 64) vectors; method 1 = the 4th-order
 * Runge-Kutta update (eqs. runge kutta 1-4, runge kutta), m_max and tol
 * unused; method 2 = the Taylor expansion of exp(-i dt H/hbar) to order
 * m_max (Section 3.1 runs order 2): T_0 = psi, T_k = (-i dt/hbar / k) H
 * T_{k-1}, each term compressed, psi(t + dt) = sum_k T_k compressed; tol
 * unused.  H x is the exact MPO x MPS product; a compression orthonormalises
 * left to right (every singular value kept) and truncates right to left with
 * the DBSS rule of the sweep (eps, D_max, capped at the MPS capacity).  Unlike the
 * local steps this grows bonds through couplings of any range (the paper
 * runs global steps first for that reason) at the price of intermediates
 * with bonds D * w; an intermediate bond above 192 (the largest validated
 * one) is refused with TDMRG_EUNSUPPORTED before the step changes anything.
 * The MPS is left right-canonical with its centre on
 * site 0.  stats (optional): basis vectors used (4 for RK4, the order for
 * Taylor), largest
 * intermediate bond, summed discarded weight, host wall seconds. */
typedef struct {
  int vectors, max_intermediate_bond;
  double sum_disc, seconds;
} tdmrg_global_stats;
/* How the global steps apply H and form sums (Section 2.1.1):
 * mode 0 (default): the direct procedure, the exact MPO x MPS product
 *   (bonds D * w) and block sums (bonds sum_k D_k), each then compressed
 *   (intermediates above bond 192 are refused, see tdmrg_global_step);
 * mode 1: the variational procedure of eq. variational app: |phi>
 *   minimising || |phi> - sum_k c_k O_k |x_k> ||^2 (O_k = H for a product,
 *   the identity for a sum) by sweeping two-site updates, each the
 *   contraction of the pair of every x_k with the left and right blocks of
 *   <phi| O_k |x_k> followed by the DBSS truncation (eps, D_max); sweeps
 *   until |phi|^2 changes by at most 1e-15 relative (about its rounding
 *   level), at most 16, starting from a right-canonical copy of x_0.  No intermediate wider than D_max
 *   is formed, so no size limit applies.
 * EINVAL for another mode. */
tdmrg_status tdmrg_ctx_set_mpo_apply(tdmrg_ctx* ctx, int mode);
tdmrg_status tdmrg_global_step(tdmrg_ctx* ctx, tdmrg_mps* mps, const tdmrg_mpo* mpo, double dt_fs, int method,
                               int m_max, double tol, int D_max, double eps, tdmrg_global_stats* stats);

/* Observables (Section 3.1): raw expectation values, not divided by the norm.
 *   pops[n_el] = <psi| |i><i| x 1 |psi>,  norm2 = <psi|psi>,  energy = <psi|H|psi>,
 *   (c_re, c_im) = <psi0|psi> (eqs. overlap 1/2) when psi0 != NULL (else 0),
 *   mps_size = sum_i m_{i-1} d_i m_i.
 * pops is host memory of n_el doubles supplied by the caller. */
/* ---- gradient of a whole evolution --------------------------------------
 * Gradient of P_state(T) = <psi(T)| |state><state| (x) 1 |psi(T)> after
 * `steps` symmetric 2TDVP steps (as tdmrg_tdvp2_sweep, FP64) from the
 * product state occ, with respect to the coupling constants of the model
 * (eqs. Hel_2, Hvib_2, Helvib_2), at the truncation ranks the forward run
 * chose.  Reverse mode over the whole evolution: per-step checkpoints of
 * the sites and right environments, the step recomputed from its
 * checkpoint, then the adjoints of the one-site and two-site exponentials
 * (Frechet integral by Gauss-Legendre quadrature with at most nquad nodes:
 * per exponential, the fewest nodes whose error bound for the spectral
 * spread of its Krylov tridiagonals is below 1e-15), of the
 * environment updates, of the truncated SVD (the gauge-invariant part,
 * through the derivative of the kept singular subspace, from a full SVD)
 * and of the two-site tensor formation; finally the MPO cotangents are
 * contracted with the (exact, since the MPO is affine in each constant)
 * MPO differences.  Every output array is optional (NULL skips it):
 * E [n_el]; V [n_el*n_el] symmetric (one constant per pair i < j, diagonal
 * zero); omega [n_modes]; g1 [n_modes*n_el*n_el] symmetric in (i, j) (one
 * constant per i <= j); g2 [n_g2].  ranks [steps][2][n_sites-1] (optional)
 * receives the kept rank of every SVD (left-to-right pairs, then
 * right-to-left pairs, by pair index).  EUNSUPPORTED for FP32 options;
 * ENOCONV when a local exponential misses the Lanczos tolerance. */
typedef struct {
  double *E, *V, *omega, *g1, *g2;
} tdmrg_model_grad;
typedef struct {
  double pop;              /* P_state(T) */
  double seconds_forward;  /* forward evolution with checkpoints */
  double seconds_total;    /* forward + reverse + parameter contraction */
  double mean_nodes;       /* quadrature nodes per exponential adjoint */
} tdmrg_grad_info;
tdmrg_status tdmrg_tdvp2_population_grad(tdmrg_ctx* ctx, const tdmrg_model* model, const int* occ, int D_cap,
                                         int steps, double dt_fs, int D_max, double eps, const tdmrg_opts* opts,
                                         int state, int nquad, tdmrg_model_grad* grad, int* ranks,
                                         tdmrg_grad_info* info);

typedef struct {
  double* pops;
  double norm2, energy, c_re, c_im, mps_size;
} tdmrg_obs;
tdmrg_status tdmrg_observables(tdmrg_ctx* ctx, const tdmrg_mps* mps, const tdmrg_mpo* mpo,
                               const tdmrg_mps* psi0, tdmrg_obs* obs);

#ifdef __cplusplus
}
#endif
#endif /* TDMRG_H */
