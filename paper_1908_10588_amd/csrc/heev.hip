// Hermitian eigensolver of the Rayleigh-Ritz step of the subspace SVD and of
// the Gram route (the eigenpairs of C = Z^H Z or theta theta^H, n <= 512):
//   1. Householder reduction to real symmetric tridiagonal form T = Q^H C Q,
//      Q = H_0 H_1 ... H_{n-2}, H_j = I - tau_j v_j v_j^H acting on rows
//      j+1..n-1 (the elementary reflector of LAPACK's zlarfg convention:
//      H_j^H x = beta e_1 with beta real), in ONE workgroup;
//   2. the eigenpairs T = Z diag(lambda) Z^T (rocSOLVER's divide and conquer
//      dstedc on the real tridiagonal matrix);
//   3. the eigenvectors of C as Q Z: every workgroup applies all reflectors,
//      last first, to a block of columns of Z held in LDS.
//
// The reduction runs as one workgroup of 1024 threads because every step
// depends on the previous one through a full pass over the trailing block:
// with the whole block in one CU, a step costs workgroup barriers only, where
// a multi-workgroup reduction would pay a device-wide synchronisation per
// step.  Each step makes ONE pass over the trailing block: it applies the
// previous step's rank-2 update A <- A - v w^H - w v^H while forming the
// product p = tau A v of the current step (one read and one write per
// element).  The trailing block lives in L2-resident global memory until it
// fits LDS (order <= 80), after which the remaining steps run from LDS.
#include <math.h>

#include "kernels.h"

namespace tdmrg {

namespace {

constexpr int TRD_THREADS = 1024;
constexpr int TRD_WAVES = TRD_THREADS / 64;
constexpr int TRD_LDS = 80;  // order of the trailing block held in LDS
constexpr int TRD_BATCH = 8;  // rows of the trailing block loaded together

// Cross-lane moves of a double by DPP (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of x over each row of 16 lanes, in every lane of the row: quad
// permutations (lane ^ 1, lane ^ 2) and row rotations by 4 and 8.
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_d<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_d<0x124>(x);  // row_ror:4
  x += dpp_d<0x128>(x);  // row_ror:8
  return x;
}

// Sum over the wave, the same value in every lane (rows added in order).
__device__ __forceinline__ double wave_sum(double x) {
  x = row16_sum(x);
  return (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
}

// Workgroup barrier that orders LDS accesses only: global stores before it
// are not waited for (use __syncthreads where another wave reads them).
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over the workgroup of (a, b), in a fixed order (waves 0..15).  red
// must not be reused by the next call before a barrier (callers alternate two).
__device__ __forceinline__ void block_sum2(double& a, double& b, double (*red)[TRD_WAVES]) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
  }
  lds_sync();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < TRD_WAVES; ++w) {
    sa += red[0][w];
    sb += red[1][w];
  }
  a = sa;
  b = sb;
}

// One pass over the trailing block of step j (rows and columns j+1..n-1;
// element (j+1+c, j+1+r) at Ar/Ai[base + c * ld + r]).  Wave w takes column
// block r in [64 cb, 64 cb + 64) (lane = column) and a slice of the rows c,
// so every load is a contiguous row segment and no cross-lane sums are needed:
//   a <- a - v'_{c+1} conj(w'_{r+1}) - w'_{c+1} conj(v'_{r+1})  (step j-1's update, when pending)
//   part_r += conj(a) v_c          (= A[r][c] v_c: the block is Hermitian)
// The partial sums of each wave land in part[wave][lane]; the updated first
// column of the block (the next step's diagonal and column) in col[c].
template <typename P>
__device__ __forceinline__ void trailing_pass(P Ar, P Ai, long ld, int off, int j, int m, bool pending,
                                              const double* vpr, const double* vpi, const double* wpr,
                                              const double* wpi, const double* vr, const double* vi,
                                              double* partr, double* parti, double* colr, double* coli) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ncb = (m + 63) >> 6;
  const int S = TRD_WAVES / ncb;  // row slices per column block
  const int cb = wave / S, rs = wave - cb * S;
  const int r = cb * 64 + lane;
  double sr = 0.0, si = 0.0;
  if (cb < ncb && r < m) {
    const long base = (long)(j + 1 - off) * ld + (j + 1 - off) + r;
    const int per = (m + S - 1) / S;
    const int c0 = rs * per, c1 = min(m, c0 + per);
    const double bvr = pending ? vpr[r + 1] : 0.0, bvi = pending ? vpi[r + 1] : 0.0;
    const double bwr = pending ? wpr[r + 1] : 0.0, bwi = pending ? wpi[r + 1] : 0.0;
    // rows in batches of TRD_BATCH: all loads of a batch are issued before its
    // stores, so that they are in flight together
    for (int cb0 = c0; cb0 < c1; cb0 += TRD_BATCH) {
      double xr[TRD_BATCH], xi[TRD_BATCH];
#pragma unroll
      for (int b = 0; b < TRD_BATCH; ++b) {
        const long o = base + (long)(cb0 + b) * ld;
        xr[b] = cb0 + b < c1 ? Ar[o] : 0.0;
        xi[b] = cb0 + b < c1 ? Ai[o] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < TRD_BATCH; ++b) {
        const int c = cb0 + b;
        if (c < c1) {
          double ar = xr[b], ai = xi[b];
          if (pending) {
            const double avr = vpr[c + 1], avi = vpi[c + 1], awr = wpr[c + 1], awi = wpi[c + 1];
            // v_c conj(w_r) + w_c conj(v_r)
            ar -= (avr * bwr + avi * bwi) + (awr * bvr + awi * bvi);
            ai -= (avi * bwr - avr * bwi) + (awi * bvr - awr * bvi);
            const long o = base + (long)c * ld;
            Ar[o] = ar;
            Ai[o] = ai;
          }
          if (r == 0) {
            colr[c] = ar;
            coli[c] = ai;
          }
          const double ur = vr[c], ui = vi[c];
          sr += ar * ur + ai * ui;
          si += ar * ui - ai * ur;
        }
      }
    }
  }
  partr[wave * 64 + lane] = sr;
  parti[wave * 64 + lane] = si;
}

}  // namespace

// C: planar row-major n x n Hermitian (plane offset n*n; the lower triangle
// is read, the diagonal's real part).  A: scratch [2][n][n].  V: [2][n][n],
// row j = v_j (v_j[0] = 1, m = n-1-j entries).  d[n], e[n-1]: the
// tridiagonal matrix.  tau: [2][n].
__global__ __launch_bounds__(TRD_THREADS) void hetrd_kernel(const double* __restrict__ C, int n,
                                                            double* __restrict__ A, double* __restrict__ V,
                                                            double* __restrict__ d, double* __restrict__ e,
                                                            double* __restrict__ tau) {
  __shared__ double sAr[TRD_LDS * TRD_LDS], sAi[TRD_LDS * TRD_LDS];
  __shared__ double vr[2][kHeevMax], vi[2][kHeevMax];  // current and pending reflector
  __shared__ double wr[kHeevMax], wi[kHeevMax];        // pending update vector
  __shared__ double xr_[kHeevMax], xi_[kHeevMax];      // column j with the pending update
  __shared__ double colr[kHeevMax], coli[kHeevMax];    // first column of the last pass's block
  __shared__ double partr[TRD_THREADS], parti[TRD_THREADS];
  __shared__ double red[2][2][TRD_WAVES];
  const int tid = threadIdx.x;
  const long nn = (long)n * n;
  const int L = n < TRD_LDS ? n : TRD_LDS;
  const int jL = n - L;  // first row and column of the LDS block
  double* Ar = A;
  double* Ai = A + nn;

  // symmetrised copy of C: A[i][k] = C[i][k] (i > k), conj(C[k][i]) (i < k), Re C[i][i]
  for (long t = tid; t < nn; t += TRD_THREADS) {
    const int i = (int)(t / n), k = (int)(t - (long)i * n);
    double xr, xi;
    if (i > k) {
      xr = C[t];
      xi = C[nn + t];
    } else if (i < k) {
      const long s = (long)k * n + i;
      xr = C[s];
      xi = -C[nn + s];
    } else {
      xr = C[t];
      xi = 0.0;
    }
    if (jL == 0) {
      sAr[i * L + k] = xr;
      sAi[i * L + k] = xi;
    } else {
      Ar[t] = xr;
      Ai[t] = xi;
    }
  }
  __syncthreads();

  int cur = 0;
  for (int j = 0; j + 1 < n; ++j) {
    const int m = n - 1 - j;
    const bool pending = j > 0;
    const double* vpr = vr[cur ^ 1];
    const double* vpi = vi[cur ^ 1];
    if (j + 1 == jL) {  // the trailing block from here on fits LDS
      for (int t = tid; t < L * L; t += TRD_THREADS) {
        const int i = t / L, k = t - i * L;
        const long g = (long)(jL + i) * n + (jL + k);
        sAr[t] = Ar[g];
        sAi[t] = Ai[g];
      }
      lds_sync();
    }
    const bool col_lds = j >= jL;             // column j (and the diagonal j) in the LDS block
    const bool col_cap = j > 0 && j < jL;     // ... else captured by step j-1's pass over global memory
    // (a) x = column j below the diagonal, with step j-1's update
    double part = 0.0, dummy = 0.0;
    for (int t = tid; t < m; t += TRD_THREADS) {
      double xr, xi;
      if (col_lds) {
        const int o = (j + 1 + t - jL) * L + (j - jL);
        xr = sAr[o];
        xi = sAi[o];
      } else if (col_cap) {
        xr = colr[t + 1];
        xi = coli[t + 1];
      } else {
        const long o = (long)(j + 1 + t) * n + j;
        xr = Ar[o];
        xi = Ai[o];
      }
      if (pending) {  // pending indices (t+1, 0)
        const double a_r = vpr[t + 1], a_i = vpi[t + 1], b_r = wr[t + 1], b_i = wi[t + 1];
        xr -= (a_r * wr[0] + a_i * wi[0]) + (b_r * vpr[0] + b_i * vpi[0]);
        xi -= (a_i * wr[0] - a_r * wi[0]) + (b_i * vpr[0] - b_r * vpi[0]);
      }
      xr_[t] = xr;
      xi_[t] = xi;
      if (t > 0) part += xr * xr + xi * xi;
    }
    if (tid == 0) {  // the diagonal j is final once step j-1's update is applied
      double a = col_lds ? sAr[(j - jL) * L + (j - jL)] : (col_cap ? colr[0] : Ar[(long)j * n + j]);
      if (pending) a -= 2.0 * (vpr[0] * wr[0] + vpi[0] * wi[0]);
      d[j] = a;
    }
    block_sum2(part, dummy, red[0]);  // barrier: x complete
    const double xnorm2 = part;
    // (b) reflector: H^H (alpha, x) = (beta, 0), H = I - tau v v^H, v_0 = 1
    const double alr = xr_[0], ali = xi_[0];
    double tr = 0.0, ti = 0.0, beta = alr, sr = 0.0, si = 0.0;
    const bool reflect = !(xnorm2 == 0.0 && ali == 0.0);
    if (reflect) {
      beta = -copysign(sqrt(alr * alr + ali * ali + xnorm2), alr);
      tr = (beta - alr) / beta;
      ti = -ali / beta;
      const double dr = alr - beta, den = dr * dr + ali * ali;  // 1 / (alpha - beta)
      sr = dr / den;
      si = -ali / den;
    }
    for (int t = tid; t < m; t += TRD_THREADS) {
      double ur = 1.0, ui = 0.0;
      if (t > 0) {
        const double xr = xr_[t], xi = xi_[t];
        ur = reflect ? xr * sr - xi * si : 0.0;
        ui = reflect ? xr * si + xi * sr : 0.0;
      }
      vr[cur][t] = ur;
      vi[cur][t] = ui;
      V[(long)j * n + t] = ur;
      V[nn + (long)j * n + t] = ui;
    }
    if (tid == 0) {
      tau[j] = tr;
      tau[n + j] = ti;
      e[j] = beta;
    }
    lds_sync();  // v complete
    // (c) one pass over the trailing block: step j-1's update, partial sums of A v
    if (j + 1 >= jL)
      trailing_pass(sAr, sAi, (long)L, jL, j, m, pending, vpr, vpi, wr, wi, vr[cur], vi[cur], partr, parti, colr,
                    coli);
    else
      trailing_pass(Ar, Ai, (long)n, 0, j, m, pending, vpr, vpi, wr, wi, vr[cur], vi[cur], partr, parti, colr,
                    coli);
    lds_sync();  // partial sums complete; step j-1's w no longer read
    // (d) p = tau A v (the row slices summed in order), w = p - (c / 2) v with
    // c = conj(tau) v^H p (real)
    const int ncb = (m + 63) >> 6, S = TRD_WAVES / ncb;
    double p_r = 0.0, p_i = 0.0, hr = 0.0, hi = 0.0;
    if (tid < m) {
      const int cb = tid >> 6, l = tid & 63;
      double qr = 0.0, qi = 0.0;
      for (int q = 0; q < S; ++q) {
        qr += partr[(cb * S + q) * 64 + l];
        qi += parti[(cb * S + q) * 64 + l];
      }
      p_r = tr * qr - ti * qi;
      p_i = tr * qi + ti * qr;
      const double ur = vr[cur][tid], ui = vi[cur][tid];
      hr = ur * p_r + ui * p_i;
      hi = ur * p_i - ui * p_r;
    }
    block_sum2(hr, hi, red[1]);
    const double c2 = 0.5 * (tr * hr + ti * hi);
    if (tid < m) {
      wr[tid] = p_r - c2 * vr[cur][tid];
      wi[tid] = p_i - c2 * vi[cur][tid];
    }
    // w complete; after a pass over global memory also its stores, which
    // other waves read in the next step
    if (j + 1 < jL)
      __syncthreads();
    else
      lds_sync();
    cur ^= 1;
  }
  if (tid == 0) {  // last diagonal: step n-2's update (pending indices (0, 0))
    double a = sAr[(n - 1 - jL) * L + (n - 1 - jL)];
    if (n > 1) a -= 2.0 * (vr[cur ^ 1][0] * wr[0] + vi[cur ^ 1][0] * wi[0]);
    d[n - 1] = a;
    if (n == 1) e[0] = 0.0;
  }
}

hipError_t launch_hetrd(const double* C, int n, double* A, double* V, double* d, double* e, double* tau,
                        hipStream_t s) {
  if (n < 1 || n > kHeevMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hetrd_kernel, dim3(1), dim3(TRD_THREADS), 0, s, C, n, A, V, d, e, tau);
  return hipGetLastError();
}

// ------------------------------------------------------ back-transformation --
constexpr int UM_COLS = 8;     // output columns per workgroup (32 lanes each)
constexpr int UM_STAGE = 8;    // reflectors staged in LDS at a time

// Eigenvectors of C = Q Z for the k largest eigenvalues (largest first):
// output column j is Q z_{n-1-j}, with z the columns of the column-major n x n
// real Z (ascending eigenvalues).  transpose = 0: out[i * k + j]; 1:
// out[j * n + i]; conj = 1 conjugates.  out's imaginary plane at out + n * k.
__global__ __launch_bounds__(256) void unmtr_kernel(const double* __restrict__ V, const double* __restrict__ tau,
                                                    const double* __restrict__ Z, int n, int k, int transpose,
                                                    int conj, double* __restrict__ out) {
  __shared__ double Wr[UM_COLS][kHeevMax], Wi[UM_COLS][kHeevMax];
  __shared__ double Sr[UM_STAGE][kHeevMax], Si[UM_STAGE][kHeevMax];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * UM_COLS;
  const long nn = (long)n * n;
  for (int t = tid; t < n * UM_COLS; t += 256) {
    const int c = t / n, i = t - c * n;
    const int j = c0 + c;
    Wr[c][i] = j < k ? Z[(long)(n - 1 - j) * n + i] : 0.0;
    Wi[c][i] = 0.0;
  }
  const int c = tid >> 5, l = tid & 31;
  const bool half = (tid & 63) >= 32;
  // reflectors n-2 down to 0, staged UM_STAGE at a time
  for (int hi = n - 2; hi >= 0; hi -= UM_STAGE) {
    const int lo = hi - UM_STAGE + 1 < 0 ? 0 : hi - UM_STAGE + 1;
    lds_sync();  // previous stage consumed (and W loaded)
    for (int s = 0; s <= hi - lo; ++s) {
      const int jr = hi - s, m = n - 1 - jr;
      for (int i = tid; i < m; i += 256) {
        Sr[s][i] = V[(long)jr * n + i];
        Si[s][i] = V[nn + (long)jr * n + i];
      }
    }
    lds_sync();
    for (int s = 0; s <= hi - lo; ++s) {
      const int jr = hi - s, m = n - 1 - jr;
      const double tr = tau[jr], ti = tau[n + jr];
      // y = v^H W[jr+1.., c]
      double yr = 0.0, yi = 0.0;
      for (int i = l; i < m; i += 32) {
        const double ar = Sr[s][i], ai = Si[s][i];
        const double xr = Wr[c][jr + 1 + i], xi = Wi[c][jr + 1 + i];
        yr += ar * xr + ai * xi;
        yi += ar * xi - ai * xr;
      }
      // sums over each half-wave (rows of 16 lanes added in order)
      yr = row16_sum(yr);
      yi = row16_sum(yi);
      yr = half ? readlane_d(yr, 32) + readlane_d(yr, 48) : readlane_d(yr, 0) + readlane_d(yr, 16);
      yi = half ? readlane_d(yi, 32) + readlane_d(yi, 48) : readlane_d(yi, 0) + readlane_d(yi, 16);
      // W[jr+1.., c] -= tau v y   (each column is owned by its 32 lanes)
      const double gr = tr * yr - ti * yi, gi = tr * yi + ti * yr;
      for (int i = l; i < m; i += 32) {
        const double ar = Sr[s][i], ai = Si[s][i];
        Wr[c][jr + 1 + i] -= ar * gr - ai * gi;
        Wi[c][jr + 1 + i] -= ar * gi + ai * gr;
      }
    }
  }
  lds_sync();
  const double sg = conj ? -1.0 : 1.0;
  const long plane = (long)n * k;
  for (int t = tid; t < n * UM_COLS; t += 256) {
    int i, cc;
    if (transpose) {  // out[j][i]: consecutive threads along i
      cc = t / n;
      i = t - cc * n;
    } else {
      i = t / UM_COLS;
      cc = t - i * UM_COLS;
    }
    const int j = c0 + cc;
    if (j >= k) continue;
    const long o = transpose ? (long)j * n + i : (long)i * k + j;
    out[o] = Wr[cc][i];
    out[plane + o] = sg * Wi[cc][i];
  }
}

hipError_t launch_unmtr(const double* V, const double* tau, const double* Z, int n, int k, int transpose, int conj,
                        double* out, hipStream_t s) {
  if (n < 1 || n > kHeevMax || k < 1 || k > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(unmtr_kernel, dim3((k + UM_COLS - 1) / UM_COLS), dim3(256), 0, s, V, tau, Z, n, k, transpose,
                     conj, out);
  return hipGetLastError();
}

}  // namespace tdmrg
