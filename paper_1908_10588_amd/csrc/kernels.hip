// HIP kernels of the tdmrg library for gfx950 (CDNA4, wave64), apart from
// the complex GEMM:
// * mix:    the block-sparse MPO channel stages (CSR over output rows).
// * Lanczos vector kernels with fixed-order (deterministic) reductions and a
//   one-wave symmetric tridiagonal eigensolver for exp(-i tau T) e1.
// * SVD packing / DBSS rank selection helpers, a one-workgroup one-sided
//   Jacobi SVD, and the pieces of the subspace-iteration truncated SVD.
#include "kernels.h"

#include <math.h>
#include <stdint.h>

#include <algorithm>

namespace tdmrg {
// ------------------------------------------------------------------ mixing --
__device__ __forceinline__ void mix_one(const MixArgs& a, long idx) {
  {
    const int q = (int)(idx % a.Q);
    long t = idx / a.Q;
    const int p = (int)(t % a.P);
    t /= a.P;
    const int srow = (int)(t % a.dout);
    const int c = (int)(t / a.dout);
    const int row = c * a.dout + srow;
    double accr = 0.0, acci = 0.0;
    const int e1 = a.rowptr[row + 1];
    for (int e = a.rowptr[row]; e < e1; ++e) {
      const int ws = a.col[e];
      const int w = ws / a.din, sp = ws - w * a.din;
      const long off = (((long)w * a.P + p) * a.din + sp) * a.Q + q;
      const double xr = a.in[off], xi = a.in[a.in_im + off];
      const double vr = a.vre[e], vi = a.vim[e];
      accr += vr * xr - vi * xi;
      acci += vr * xi + vi * xr;
    }
    const long o = (((long)c * a.P + p) * a.dout + srow) * a.Q + q;
    a.out[o] = accr;
    a.out[a.out_im + o] = acci;
  }
}

__global__ __launch_bounds__(256) void mix_kernel(MixArgs a) {
  const long total = (long)a.nout * a.dout * a.P * a.Q;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x)
    mix_one(a, idx);
}

// All problems of a batch in one launch: elem_start[p] is the first output
// element of problem p (elem_start[np] = total).  Each block finds the problem
// of its first element once; threads step forward across problem boundaries.
__global__ __launch_bounds__(256) void mix_grouped_kernel(const MixArgs* __restrict__ args,
                                                          const long* __restrict__ elem_start, int np) {
  const long total = elem_start[np];
  __shared__ int s_p;
  for (long base = (long)blockIdx.x * blockDim.x; base < total; base += (long)gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = np - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (elem_start[mid] <= base) lo = mid;
        else hi = mid - 1;
      }
      s_p = lo;
    }
    __syncthreads();
    const long idx = base + threadIdx.x;
    int p = s_p;
    __syncthreads();
    if (idx < total) {
      while (p + 1 < np && elem_start[p + 1] <= idx) ++p;
      mix_one(args[p], idx - elem_start[p]);
    }
  }
}

hipError_t launch_mix_grouped(const MixArgs* args_dev, const long* elem_start_dev, int np, long total,
                              hipStream_t s) {
  if (np <= 0 || total <= 0) return hipSuccess;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(mix_grouped_kernel, dim3((unsigned)blocks), dim3(256), 0, s, args_dev, elem_start_dev,
                     np);
  return hipGetLastError();
}

// One output row (channel c, local index srow) and one chunk of the
// contiguous (p, q) span per workgroup, threads over the chunk: no 64-bit
// index decoding, and the row's CSR entries are decoded once per chunk into
// LDS offsets shared by the block.  Same summation order per output element
// as mix_one.  Workgroups are numbered so that each XCD (hardware ids are
// dealt round-robin over the 8) receives a contiguous range, and within it
// consecutive ids run over the rows of one chunk: the input rows that
// neighbouring output rows share (the channel operators are banded in the
// local indices) are then re-read from that XCD's L2.
constexpr int MIXR_THREADS = 256;

template <typename S>
__global__ __launch_bounds__(MIXR_THREADS) void mix_rows_kernel(MixArgs a, long nrows) {
  const S* in = (const S*)a.in;
  S* out = (S*)a.out;
  __shared__ long s_off[MIXR_THREADS];
  __shared__ double s_vr[MIXR_THREADS], s_vi[MIXR_THREADS];
  const long nb = gridDim.x, b = blockIdx.x;
  const long q8 = nb / 8, r8 = nb % 8, xcd = b % 8, slot = b / 8;
  const long id = (xcd < r8) ? xcd * (q8 + 1) + slot : r8 * (q8 + 1) + (xcd - r8) * q8 + slot;
  const int row = (int)(id % nrows);
  const long chunk = id / nrows;
  const long PQ = (long)a.P * a.Q;
  const long pq = chunk * MIXR_THREADS + threadIdx.x;
  const bool act = pq < PQ;
  const int p = act ? (int)(pq / a.Q) : 0;
  const int q = act ? (int)(pq - (long)p * a.Q) : 0;
  const long base = (long)p * a.din * a.Q + q;
  const long wstride = (long)a.P * a.din * a.Q;
  double accr = 0.0, acci = 0.0;
  const int e0 = a.rowptr[row], e1 = a.rowptr[row + 1];
  for (int c0 = e0; c0 < e1; c0 += MIXR_THREADS) {
    const int n = min(MIXR_THREADS, e1 - c0);
    __syncthreads();  // the previous chunk has been consumed
    if ((int)threadIdx.x < n) {
      const int ws = a.col[c0 + threadIdx.x];
      const int w = ws / a.din, sp = ws - w * a.din;
      s_off[threadIdx.x] = (long)w * wstride + (long)sp * a.Q;
      s_vr[threadIdx.x] = a.vre[c0 + threadIdx.x];
      s_vi[threadIdx.x] = a.vim[c0 + threadIdx.x];
    }
    __syncthreads();
    if (act) {
      int e = 0;
      // four entries' loads in flight at once; accumulation stays in entry order
      for (; e + 4 <= n; e += 4) {
        double xr[4], xi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long off = base + s_off[e + u];
          xr[u] = in[off];
          xi[u] = in[a.in_im + off];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double vr = s_vr[e + u], vi = s_vi[e + u];
          accr += vr * xr[u] - vi * xi[u];
          acci += vr * xi[u] + vi * xr[u];
        }
      }
      for (; e < n; ++e) {
        const long off = base + s_off[e];
        const double xr = in[off], xi = in[a.in_im + off];
        const double vr = s_vr[e], vi = s_vi[e];
        accr += vr * xr - vi * xi;
        acci += vr * xi + vi * xr;
      }
    }
  }
  if (act) {
    const int c = row / a.dout, srow = row - c * a.dout;
    const long o = (((long)c * a.P + p) * a.dout + srow) * a.Q + q;
    out[o] = (S)accr;
    out[a.out_im + o] = (S)acci;
  }
}

// Several output rows per workgroup: kMixRows consecutive rows (their
// distinct input columns staged in LDS with each row's coefficient) over a
// chunk of 512 elements of the contiguous (p, q) span, two neighbouring q per
// thread in 16-byte loads.  Every input element a block needs is read once
// per block instead of once per row that uses it (the channel operators are
// banded in the local indices, so consecutive rows share most columns).  Per
// output element the entries are summed in ascending column order with the
// same expressions as the one-row kernel, so both give the same bits.
constexpr int MIXB_THREADS = 256;
constexpr int MIXB_STAGE = 128;  // columns staged in LDS per pass
// columns whose loads are issued together (FP64: 4, at four waves per SIMD; FP32: 8)
template <typename S>
constexpr int mixb_inflight() { return sizeof(S) == 4 ? 8 : 4; }

template <typename S> struct Pair2;
template <> struct Pair2<double> { typedef double2 type; };
template <> struct Pair2<float> { typedef float2 type; };

template <typename S>
__global__ __launch_bounds__(MIXB_THREADS) void mix_block_kernel(MixArgs a, long nblk, long nrows) {
  typedef typename Pair2<S>::type S2;
  const S* in = (const S*)a.in;
  S* out = (S*)a.out;
  __shared__ long s_off[MIXB_STAGE];
  __shared__ unsigned s_mask[MIXB_STAGE];
  __shared__ double s_vr[MIXB_STAGE][kMixRows], s_vi[MIXB_STAGE][kMixRows];
  const long nb = gridDim.x, b = blockIdx.x;
  const long q8 = nb / 8, r8 = nb % 8, xcd = b % 8, slot = b / 8;
  const long id = (xcd < r8) ? xcd * (q8 + 1) + slot : r8 * (q8 + 1) + (xcd - r8) * q8 + slot;
  const long B = id % nblk;
  const long chunk = id / nblk;
  const long PQ = (long)a.P * a.Q;
  const long e = 2 * (chunk * MIXB_THREADS + threadIdx.x);  // first of this thread's two elements
  const bool act = e < PQ;
  const int p = act ? (int)(e / a.Q) : 0;
  const int q = act ? (int)(e - (long)p * a.Q) : 0;  // even: Q is even
  const long base = (long)p * a.din * a.Q + q;
  const long wstride = (long)a.P * a.din * a.Q;
  double ar0[kMixRows], ar1[kMixRows], ai0[kMixRows], ai1[kMixRows];
#pragma unroll
  for (int r = 0; r < kMixRows; ++r) ar0[r] = ar1[r] = ai0[r] = ai1[r] = 0.0;
  const int u0 = a.blk.bptr[B], u1 = a.blk.bptr[B + 1];
  for (int c0 = u0; c0 < u1; c0 += MIXB_STAGE) {
    const int n = min(MIXB_STAGE, u1 - c0);
    __syncthreads();  // the previous columns have been consumed
    if ((int)threadIdx.x < n) {
      const int t = threadIdx.x, ws = a.blk.bcol[c0 + t];
      const int w = ws / a.din, sp = ws - w * a.din;
      s_off[t] = (long)w * wstride + (long)sp * a.Q;
      s_mask[t] = a.blk.bmask[c0 + t];
#pragma unroll
      for (int r = 0; r < kMixRows; ++r) {
        s_vr[t][r] = a.blk.bval[(long)(c0 + t) * kMixRows + r];
        s_vi[t][r] = a.blk.bval[(a.blk.ncols + c0 + t) * kMixRows + r];
      }
    }
    __syncthreads();
    if (act) {
      int u = 0;
      constexpr int NF = mixb_inflight<S>();
      for (; u + NF <= n; u += NF) {  // several columns' loads in flight
        S2 xr[NF], xi[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          const long off = base + s_off[u + k];
          xr[k] = *(const S2*)(in + off);
          xi[k] = *(const S2*)(in + a.in_im + off);
        }
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          const unsigned m = __builtin_amdgcn_readfirstlane(s_mask[u + k]);
#pragma unroll
          for (int r = 0; r < kMixRows; ++r)
            if (m >> r & 1u) {
              const double vr = s_vr[u + k][r], vi = s_vi[u + k][r];
              const double x0 = xr[k].x, y0 = xi[k].x, x1 = xr[k].y, y1 = xi[k].y;
              ar0[r] += vr * x0 - vi * y0;
              ai0[r] += vr * y0 + vi * x0;
              ar1[r] += vr * x1 - vi * y1;
              ai1[r] += vr * y1 + vi * x1;
            }
        }
      }
      for (; u < n; ++u) {
        const long off = base + s_off[u];
        const S2 xr = *(const S2*)(in + off), xi = *(const S2*)(in + a.in_im + off);
        const double x0 = xr.x, y0 = xi.x, x1 = xr.y, y1 = xi.y;
        const unsigned m = __builtin_amdgcn_readfirstlane(s_mask[u]);
#pragma unroll
        for (int r = 0; r < kMixRows; ++r)
          if (m >> r & 1u) {
            const double vr = s_vr[u][r], vi = s_vi[u][r];
            ar0[r] += vr * x0 - vi * y0;
            ai0[r] += vr * y0 + vi * x0;
            ar1[r] += vr * x1 - vi * y1;
            ai1[r] += vr * y1 + vi * x1;
          }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < kMixRows; ++r) {
      const long row = B * kMixRows + r;
      if (row >= nrows) break;
      const int c = (int)(row / a.dout), srow = (int)(row - (long)c * a.dout);
      const long o = (((long)c * a.P + p) * a.dout + srow) * a.Q + q;
      *(S2*)(out + o) = S2{(S)ar0[r], (S)ar1[r]};
      *(S2*)(out + a.out_im + o) = S2{(S)ai0[r], (S)ai1[r]};
    }
  }
}

hipError_t launch_mix(const MixArgs& a, hipStream_t s) {
  const long rows = (long)a.nout * a.dout;
  const long PQ = (long)a.P * a.Q;
  if (rows <= 0 || PQ <= 0) return hipSuccess;
  // two-element loads and stores need an even q span and even plane offsets
  // on arrays aligned to two elements
  const uintptr_t al = a.f32 ? 7 : 15;
  const bool pairs = a.blk.bptr && a.Q % 2 == 0 && a.in_im % 2 == 0 && a.out_im % 2 == 0 &&
                     ((uintptr_t)a.in & al) == 0 && ((uintptr_t)a.out & al) == 0;
  if (pairs) {
    const long nblk = (rows + kMixRows - 1) / kMixRows;
    const long chunks = (PQ / 2 + MIXB_THREADS - 1) / MIXB_THREADS;
    if (nblk * chunks <= 0x7fffffffL) {
      if (a.f32)
        hipLaunchKernelGGL(mix_block_kernel<float>, dim3((unsigned)(nblk * chunks)), dim3(MIXB_THREADS), 0, s, a,
                           nblk, rows);
      else
        hipLaunchKernelGGL(mix_block_kernel<double>, dim3((unsigned)(nblk * chunks)), dim3(MIXB_THREADS), 0, s, a,
                           nblk, rows);
      return hipGetLastError();
    }
  }
  const long bx = (PQ + MIXR_THREADS - 1) / MIXR_THREADS;
  if (bx * rows <= 0x7fffffffL) {
    if (a.f32)
      hipLaunchKernelGGL(mix_rows_kernel<float>, dim3((unsigned)(bx * rows)), dim3(MIXR_THREADS), 0, s, a, rows);
    else
      hipLaunchKernelGGL(mix_rows_kernel<double>, dim3((unsigned)(bx * rows)), dim3(MIXR_THREADS), 0, s, a, rows);
    return hipGetLastError();
  }
  if (a.f32) return hipErrorInvalidValue;  // the element-wise fallback reads FP64 only
  const long total = (long)a.nout * a.dout * a.P * a.Q;
  if (total <= 0) return hipSuccess;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(mix_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------- Lanczos vectors ----
constexpr int DOT_THREADS = 256;
constexpr int DOT_JB = 4;  // Krylov vectors per block row
constexpr int DOT_MAX_CHUNKS = 1024;

int dot_chunks(long n) {
  long c = (n + 4L * DOT_THREADS - 1) / (4L * DOT_THREADS);
  if (c < 1) c = 1;
  if (c > DOT_MAX_CHUNKS) c = DOT_MAX_CHUNKS;
  return (int)c;
}

static dim3 stream_grid(long n) {
  long b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// grid: (nchunk, ceil(nv / DOT_JB)); each block sums its chunk for DOT_JB vectors.
// With jd (device Lanczos counter j), nv = j + 1 and the grid covers the
// largest count; block rows beyond nv exit at once.
__global__ __launch_bounds__(DOT_THREADS) void multidot_kernel(const double* V, long vstride, int nv,
                                                               long n, const double* w,
                                                               double* part_re, double* part_im,
                                                               const int* jd, int nv_min) {
  if (jd) nv = *jd + 1;
  if (nv < nv_min) return;  // the fused Gram-Schmidt kernel covers small counts
  const int nchunk = gridDim.x;
  const int b = blockIdx.x;
  const int j0 = blockIdx.y * DOT_JB;
  if (j0 >= nv) return;  // uniform per block
  const long per = (n + nchunk - 1) / nchunk;
  const long lo = (long)b * per;
  const long hi = (lo + per < n) ? lo + per : n;
  double sr[DOT_JB], si[DOT_JB];
#pragma unroll
  for (int j = 0; j < DOT_JB; ++j) sr[j] = si[j] = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += DOT_THREADS) {
    const double wr = w[i], wi = w[n + i];
#pragma unroll
    for (int j = 0; j < DOT_JB; ++j) {
      if (j0 + j < nv) {
        const double* v = V + (long)(j0 + j) * vstride;
        const double vr = v[i], vi = v[n + i];
        sr[j] += vr * wr + vi * wi;  // conj(v) * w
        si[j] += vr * wi - vi * wr;
      }
    }
  }
  __shared__ double red[2][DOT_JB][DOT_THREADS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < DOT_JB; ++j) {
    const double a = wave_sum(sr[j]);
    const double c = wave_sum(si[j]);
    if (lane == 0) {
      red[0][j][wv] = a;
      red[1][j][wv] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < DOT_JB && j0 + (int)threadIdx.x < nv) {
    const int j = threadIdx.x;
    double a = 0.0, c = 0.0;
    for (int k = 0; k < DOT_THREADS / 64; ++k) {
      a += red[0][j][k];
      c += red[1][j][k];
    }
    part_re[(long)(j0 + j) * nchunk + b] = a;
    part_im[(long)(j0 + j) * nchunk + b] = c;
  }
}

hipError_t launch_multidot(const double* V, long vstride, int nv, long n, const double* w,
                           double* part_re, double* part_im, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  const int nchunk = dot_chunks(n);
  dim3 grid(nchunk, (nv + DOT_JB - 1) / DOT_JB);
  hipLaunchKernelGGL(multidot_kernel, grid, dim3(DOT_THREADS), 0, s, V, vstride, nv, n, w, part_re,
                     part_im, (const int*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_multidot_dev(const double* V, long vstride, const int* jd, int nv_max, long n, const double* w,
                               double* part_re, double* part_im, int nv_min, hipStream_t s) {
  if (nv_max <= 0 || nv_max > DOT_MAX_CHUNKS) return hipErrorInvalidValue;
  const int nchunk = dot_chunks(n);
  dim3 grid(nchunk, (nv_max + DOT_JB - 1) / DOT_JB);
  hipLaunchKernelGGL(multidot_kernel, grid, dim3(DOT_THREADS), 0, s, V, vstride, nv_max, n, w, part_re,
                     part_im, jd, nv_min);
  return hipGetLastError();
}

// one wave per vector j: lanes stride over chunks, then a fixed butterfly.
// With jd (device Lanczos counter): jmode 1 keeps blocks j <= *jd, jmode 2
// (one block) writes its result to out index *jd.
__global__ __launch_bounds__(64) void reduce_partials_kernel(const double* part_re,
                                                             const double* part_im, int nchunk,
                                                             double* out_re, double* out_im,
                                                             int mode, const int* jd, int jmode) {
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  if (jd && jmode == 1 && j > *jd) return;
  const int o = (jd && jmode == 2) ? *jd : j;
  double a = 0.0, c = 0.0;
  for (int b = lane; b < nchunk; b += 64) {
    a += part_re[(long)j * nchunk + b];
    c += part_im[(long)j * nchunk + b];
  }
  a = wave_sum(a);
  c = wave_sum(c);
  if (lane == 0) {
    if (mode == 1) {
      out_re[o] = sqrt(a > 0.0 ? a : 0.0);
    } else {
      out_re[o] = a;
      out_im[o] = c;
    }
  }
}

hipError_t launch_reduce_partials(const double* part_re, const double* part_im, int nv, int nchunk,
                                  double* out_re, double* out_im, int mode, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(nv), dim3(64), 0, s, part_re, part_im, nchunk,
                     out_re, out_im, mode, (const int*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_reduce_partials_dev(const double* part_re, const double* part_im, const int* jd, int nv_max,
                                      int nchunk, double* out_re, double* out_im, int mode, hipStream_t s) {
  if (nv_max <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(nv_max), dim3(64), 0, s, part_re, part_im, nchunk,
                     out_re, out_im, mode, jd, 1);
  return hipGetLastError();
}

constexpr int MAXV = 64;
constexpr int GS_MAXV = kGsFusedMax;  // basis vectors the fused Gram-Schmidt kernel holds in registers (8: 4 waves per SIMD; 16 left it at 2)

__global__ __launch_bounds__(256) void multiaxpy_kernel(const double* V, long vstride, int nv, long n,
                                                        const double* cr, const double* ci,
                                                        double* w, const int* jd, int nv_min) {
  if (jd) nv = *jd + 1;
  if (nv < nv_min) return;
  __shared__ double scr[MAXV], sci[MAXV];
  if (threadIdx.x < nv) {
    scr[threadIdx.x] = cr[threadIdx.x];
    sci[threadIdx.x] = ci[threadIdx.x];
  }
  __syncthreads();
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < nv; ++j) {
      const double* v = V + (long)j * vstride;
      const double vr = v[i], vi = v[n + i];
      ar += scr[j] * vr - sci[j] * vi;
      ai += scr[j] * vi + sci[j] * vr;
    }
    w[i] -= ar;
    w[n + i] -= ai;
  }
}

// w -= sum_j c_j V_j as multiaxpy, over the multidot chunking (one contiguous
// chunk per block, fixed per n), and the block's share of ||w||^2 after the
// update into part[b]: the norm needs no second pass over w.
__global__ __launch_bounds__(DOT_THREADS) void multiaxpy_norm_kernel(const double* V, long vstride, int nv,
                                                                     long n, const double* cr,
                                                                     const double* ci, double* w,
                                                                     double* part, const int* jd) {
  if (jd) nv = *jd + 1;
  __shared__ double scr[MAXV], sci[MAXV];
  __shared__ double red[DOT_THREADS / 64];
  if (threadIdx.x < nv) {
    scr[threadIdx.x] = cr[threadIdx.x];
    sci[threadIdx.x] = ci[threadIdx.x];
  }
  __syncthreads();
  const int nchunk = gridDim.x, b = blockIdx.x;
  const long per = (n + nchunk - 1) / nchunk;
  const long lo = (long)b * per;
  const long hi = (lo + per < n) ? lo + per : n;
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += DOT_THREADS) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < nv; ++j) {
      const double* v = V + (long)j * vstride;
      const double vr = v[i], vi = v[n + i];
      ar += scr[j] * vr - sci[j] * vi;
      ai += scr[j] * vi + sci[j] * vr;
    }
    const double nr = w[i] - ar, ni = w[n + i] - ai;
    w[i] = nr;
    w[n + i] = ni;
    acc += nr * nr + ni * ni;
  }
  const double a = wave_sum(acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < DOT_THREADS / 64; ++k) t += red[k];
    part[b] = t;
  }
}

hipError_t launch_multiaxpy_norm(const double* V, long vstride, int nv, long n, const double* cr,
                                 const double* ci, double* w, double* part, double* nrm, hipStream_t s) {
  if (nv > MAXV) return hipErrorInvalidValue;
  const int nchunk = dot_chunks(n);
  hipLaunchKernelGGL(multiaxpy_norm_kernel, dim3(nchunk), dim3(DOT_THREADS), 0, s, V, vstride, nv, n, cr, ci,
                     w, part, (const int*)nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_partials(part, part, 1, nchunk, nrm, nullptr, 1, s);
}

hipError_t launch_multiaxpy_norm_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                                     const double* ci, double* w, double* part, double* beta, hipStream_t s) {
  const int nchunk = dot_chunks(n);
  hipLaunchKernelGGL(multiaxpy_norm_kernel, dim3(nchunk), dim3(DOT_THREADS), 0, s, V, vstride, 0, n, cr, ci, w,
                     part, jd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(64), 0, s, (const double*)part, (const double*)part,
                     nchunk, beta, (double*)nullptr, 1, jd, 2);
  return hipGetLastError();
}

__global__ void copy_scalar_kernel(const double* src, double* dst, const int* jd) {
  if (threadIdx.x == 0) {
    const int o = jd ? *jd : 0;
    dst[o] = src[o];
  }
}

hipError_t launch_copy_scalar(const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(64), 0, s, src, dst, (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_copy_scalar_dev(const double* src, double* dst, const int* jd, hipStream_t s) {
  hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(64), 0, s, src, dst, jd);
  return hipGetLastError();
}

// End of Lanczos step j = *jd: the next basis vector w / beta_j goes to x (the
// operand of the next H product) and, when j + 1 < m_max, to V[j + 1].
__global__ __launch_bounds__(256) void lanczos_next_kernel(const double* w, long n2, const double* beta, double* V,
                                                           long vstride, double* x, const int* jd, int m_max) {
  const int j = *jd;
  const double b = beta[j];
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  double* vn = (j + 1 < m_max) ? V + (long)(j + 1) * vstride : nullptr;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    const double v = w[i] * inv;
    x[i] = v;
    if (vn) vn[i] = v;
  }
}

hipError_t launch_lanczos_next(const double* w, long n, const double* beta, double* V, long vstride, double* x,
                               const int* jd, int m_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lanczos_next_kernel, stream_grid(2 * n), dim3(256), 0, s, w, 2 * n, beta, V, vstride, x, jd,
                     m_max);
  return hipGetLastError();
}

__global__ void counter_kernel(int* c, int value, int add) {
  if (threadIdx.x == 0) c[0] = add ? c[0] + value : value;
}

hipError_t launch_counter_set(int* c, int value, hipStream_t s) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, c, value, 0);
  return hipGetLastError();
}

hipError_t launch_counter_add(int* c, int value, hipStream_t s) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, c, value, 1);
  return hipGetLastError();
}


hipError_t launch_multiaxpy(const double* V, long vstride, int nv, long n, const double* cr,
                            const double* ci, double* w, hipStream_t s) {
  if (nv <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(multiaxpy_kernel, stream_grid(n), dim3(256), 0, s, V, vstride, nv, n, cr, ci, w,
                     (const int*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_multiaxpy_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                                const double* ci, double* w, int nv_min, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(multiaxpy_kernel, stream_grid(n), dim3(256), 0, s, V, vstride, 0, n, cr, ci, w, jd, nv_min);
  return hipGetLastError();
}

// First Gram-Schmidt pass and the second pass's dots in one read of the
// basis: w -= sum_{k<nv} c_k v_k, then the partial sums of <v_k, w> on the
// updated w, with v_k held in registers between the two (nv <= GS_MAXV; for
// larger counts the kernel does nothing and the separate kernels run).
// Chunked and summed exactly as multiaxpy followed by multidot, so the
// results are bitwise theirs.
__global__ __launch_bounds__(DOT_THREADS) void gs_fused_kernel(const double* V, long vstride, long n,
                                                               const double* cr, const double* ci, double* w,
                                                               double* part_re, double* part_im, const int* jd) {
  const int nv = *jd + 1;
  if (nv > GS_MAXV) return;
  __shared__ double scr[GS_MAXV], sci[GS_MAXV];
  __shared__ double red[2][GS_MAXV][DOT_THREADS / 64];
  if ((int)threadIdx.x < nv) {
    scr[threadIdx.x] = cr[threadIdx.x];
    sci[threadIdx.x] = ci[threadIdx.x];
  }
  __syncthreads();
  const int nchunk = gridDim.x;
  const int b = blockIdx.x;
  const long per = (n + nchunk - 1) / nchunk;
  const long lo = (long)b * per;
  const long hi = (lo + per < n) ? lo + per : n;
  double dr[GS_MAXV], di[GS_MAXV];
#pragma unroll
  for (int k = 0; k < GS_MAXV; ++k) dr[k] = di[k] = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += DOT_THREADS) {
    double vr[GS_MAXV], vi[GS_MAXV];
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int k = 0; k < GS_MAXV; ++k) {
      if (k < nv) {
        const double* v = V + (long)k * vstride;
        vr[k] = v[i];
        vi[k] = v[n + i];
        ar += scr[k] * vr[k] - sci[k] * vi[k];
        ai += scr[k] * vi[k] + sci[k] * vr[k];
      }
    }
    double wr = w[i], wi = w[n + i];
    wr -= ar;
    wi -= ai;
    w[i] = wr;
    w[n + i] = wi;
#pragma unroll
    for (int k = 0; k < GS_MAXV; ++k) {
      if (k < nv) {
        dr[k] += vr[k] * wr + vi[k] * wi;  // conj(v) * w
        di[k] += vr[k] * wi - vi[k] * wr;
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < GS_MAXV; ++k) {
    if (k < nv) {
      const double a = wave_sum(dr[k]);
      const double c = wave_sum(di[k]);
      if (lane == 0) {
        red[0][k][wv] = a;
        red[1][k][wv] = c;
      }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    const int k = threadIdx.x;
    double a = 0.0, c = 0.0;
    for (int q = 0; q < DOT_THREADS / 64; ++q) {
      a += red[0][k][q];
      c += red[1][k][q];
    }
    part_re[(long)k * nchunk + b] = a;
    part_im[(long)k * nchunk + b] = c;
  }
}

hipError_t launch_gs_fused_dev(const double* V, long vstride, const int* jd, long n, const double* cr,
                               const double* ci, double* w, double* part_re, double* part_im, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gs_fused_kernel, dim3(dot_chunks(n)), dim3(DOT_THREADS), 0, s, V, vstride, n, cr, ci, w,
                     part_re, part_im, jd);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void combine_kernel(const double* V, long vstride, int nv, long n,
                                                      const double* cr, const double* ci,
                                                      const double* scale, double* out) {
  __shared__ double scr[MAXV], sci[MAXV];
  if (threadIdx.x < nv) {
    scr[threadIdx.x] = cr[threadIdx.x];
    sci[threadIdx.x] = ci[threadIdx.x];
  }
  __syncthreads();
  const double sc = scale[0];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < nv; ++j) {
      const double* v = V + (long)j * vstride;
      const double vr = v[i], vi = v[n + i];
      ar += scr[j] * vr - sci[j] * vi;
      ai += scr[j] * vi + sci[j] * vr;
    }
    out[i] = sc * ar;
    out[n + i] = sc * ai;
  }
}

hipError_t launch_combine(const double* V, long vstride, int nv, long n, const double* cr,
                          const double* ci, const double* scale_dev, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(combine_kernel, stream_grid(n), dim3(256), 0, s, V, vstride, nv, n, cr, ci,
                     scale_dev, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_inv_kernel(const double* src, long n2, const double* nrm,
                                                        double* dst) {
  const double v = nrm[0];
  const double inv = v > 0.0 ? 1.0 / v : 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i] * inv;
}

hipError_t launch_scale_by_inv(const double* src, long n, const double* nrm, double* dst,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_inv_kernel, stream_grid(2 * n), dim3(256), 0, s, src, 2 * n, nrm, dst);
  return hipGetLastError();
}

__global__ void lanczos_alpha_kernel(const double* dot_re, int j, double* alpha, const double* beta,
                                     double* cr, double* ci) {
  if (threadIdx.x == 0) {
    const double a = dot_re[0];
    alpha[j] = a;
    // coefficients ordered as the vectors [v_j, v_{j-1}]
    cr[0] = a;
    ci[0] = 0.0;
    cr[1] = (j > 0) ? beta[j - 1] : 0.0;
    ci[1] = 0.0;
  }
}

hipError_t launch_lanczos_alpha(const double* dot_re, int j, double* alpha, const double* beta,
                                double* cr, double* ci, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_alpha_kernel, dim3(1), dim3(64), 0, s, dot_re, j, alpha, beta, cr, ci);
  return hipGetLastError();
}

// One wave.  Implicit symmetric tridiagonal QR with Wilkinson shifts (Golub &
// Van Loan, Alg. 8.3.2) on d/e held in LDS; every lane evaluates the same
// rotation scalars and owns one row of the eigenvector matrix Z.  Used when
// the Chebyshev expansion below would need too many terms.
__device__ void tridiag_expm_qr(const double* alpha, const double* beta, int m, double tau, double* c_re,
                                double* c_im, double* err) {
  __shared__ double d[MAXV], e[MAXV], Z[MAXV][MAXV + 1];
  const int lane = threadIdx.x;
  if (lane < m) {
    d[lane] = alpha[lane];
    e[lane] = (lane < m - 1) ? beta[lane] : 0.0;
    for (int k = 0; k < m; ++k) Z[lane][k] = (k == lane) ? 1.0 : 0.0;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  int h = m - 1;
  int guard = 0;
  while (h > 0 && guard < 60 * m) {
    ++guard;
    if (fabs(e[h - 1]) <= eps * (fabs(d[h - 1]) + fabs(d[h]))) {
      __syncthreads();
      if (lane == 0) e[h - 1] = 0.0;
      __syncthreads();
      --h;
      continue;
    }
    int l = h - 1;
    while (l > 0 && fabs(e[l - 1]) > eps * (fabs(d[l - 1]) + fabs(d[l]))) --l;
    // Wilkinson shift from the trailing 2x2 block
    const double dd = 0.5 * (d[h - 1] - d[h]);
    const double eh = e[h - 1];
    const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * hypot(dd, eh);
    const double mu = d[h] - eh * eh / den;
    double x = d[l] - mu, z = e[l];
    double bulge = 0.0;
    for (int k = l; k < h; ++k) {
      double c, s;
      const double r = hypot(x, z);
      if (r == 0.0) {
        c = 1.0;
        s = 0.0;
      } else {
        c = x / r;
        s = -z / r;
      }
      // rotation G = [[c, s], [-s, c]] on coordinates (k, k+1): T <- G^T T G
      const double a = d[k], b = e[k], dn = d[k + 1];
      const double nd0 = a * c * c - 2.0 * b * c * s + dn * s * s;
      const double nd1 = a * s * s + 2.0 * b * c * s + dn * c * c;
      const double ne = c * s * (a - dn) + b * (c * c - s * s);
      double prev = 0.0, nbulge = 0.0, enext = 0.0;
      if (k > l) prev = e[k - 1] * c - bulge * s;  // = r
      if (k + 1 < h) {
        nbulge = -s * e[k + 1];
        enext = c * e[k + 1];
      }
      __syncthreads();
      if (lane == 0) {
        d[k] = nd0;
        d[k + 1] = nd1;
        e[k] = ne;
        if (k > l) e[k - 1] = prev;
        if (k + 1 < h) e[k + 1] = enext;
      }
      if (lane < m) {
        const double zk = Z[lane][k], zk1 = Z[lane][k + 1];
        Z[lane][k] = zk * c - zk1 * s;
        Z[lane][k + 1] = zk * s + zk1 * c;
      }
      __syncthreads();
      bulge = nbulge;
      if (k + 1 < h) {
        x = e[k];
        z = bulge;
      }
    }
  }
  __syncthreads();
  // c = Z exp(-i tau Lambda) Z^T e1
  if (lane < m) {
    double cr = 0.0, ci = 0.0;
    for (int k = 0; k < m; ++k) {
      const double ph = -tau * d[k];
      const double w0 = Z[0][k] * Z[lane][k];
      cr += w0 * cos(ph);
      ci += w0 * sin(ph);
    }
    c_re[lane] = cr;
    c_im[lane] = ci;
    if (lane == m - 1) err[0] = beta[m - 1] * hypot(cr, ci);
  }
}


// exp(-i tau T) e1 for the real symmetric tridiagonal T (diagonal alpha,
// off-diagonal beta) by the Chebyshev expansion of the exponential
// (Jacobi-Anger): with Gershgorin bounds [mu - rho, mu + rho] of the
// spectrum and X = (T - mu) / rho,
//   exp(-i tau T) = exp(-i tau mu) sum_k eps_k (-i sgn s)^k J_k(|s|) T_k(X),
// s = tau rho, eps_0 = 1, eps_k = 2.  The Bessel values J_k come from Miller's
// backward recurrence normalised by J_0 + 2 sum J_2k = 1; the vectors
// T_k(X) e1 from the three-term recurrence, one row per lane with the
// neighbours exchanged by lane shuffles.  Terms up to K = |s| + 8 |s|^(1/3)
// + 24 leave a tail below 1e-17; beyond |s| = 256 the QR route is taken.
constexpr double CHEB_ZMAX = 256.0;
constexpr int CHEB_JMAX = 400;  // > K at CHEB_ZMAX

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__global__ __launch_bounds__(64) void tridiag_expm_kernel(const double* alpha, const double* beta,
                                                          int m, double tau, double* c_re,
                                                          double* c_im, double* err, const int* jd) {
  if (jd) m = *jd + 1;  // device Lanczos counter: T_{j+1}
  __shared__ double J[CHEB_JMAX];
  const int lane = threadIdx.x;
  const bool act = lane < m;
  const double a = act ? alpha[lane] : 0.0;
  const double bl = (act && lane > 0) ? beta[lane - 1] : 0.0;   // coupling to row lane-1
  const double br = (act && lane + 1 < m) ? beta[lane] : 0.0;  // coupling to row lane+1
  const double lo = wave_min(act ? a - fabs(bl) - fabs(br) : INFINITY);
  const double hi = wave_max(act ? a + fabs(bl) + fabs(br) : -INFINITY);
  const double mu = 0.5 * (lo + hi), rho = 0.5 * (hi - lo);
  const double s = tau * rho, z = fabs(s);
  if (!isfinite(wave_sum(act ? a + bl + br : 0.0) + tau)) {  // non-finite input: NaN result
    if (act) {
      c_re[lane] = c_im[lane] = NAN;
      if (lane == m - 1) err[0] = NAN;
    }
    return;
  }
  if (!(z <= CHEB_ZMAX)) {
    tridiag_expm_qr(alpha, beta, m, tau, c_re, c_im, err);
    return;
  }
  double cr = 0.0, ci = 0.0;
  if (z == 0.0) {  // T = mu I (or tau = 0)
    cr = (lane == 0) ? 1.0 : 0.0;
  } else {
    const int K = (int)ceil(z + 8.0 * cbrt(z) + 24.0);
    const int N = K + 24 + (int)(2.0 * cbrt(z));
    if (lane == 0) {
      const double two_over_z = 2.0 / z;
      double jp = 0.0, jc = 1e-280;  // J_{k+1}, J_k (unnormalised), from k = N down
      double norm = (N % 2 == 0) ? 2.0 * jc : 0.0;
      for (int k = N; k > 0; --k) {
        const double jm = (k * two_over_z) * jc - jp;
        jp = jc;
        jc = jm;  // J_{k-1}
        if (k - 1 <= K) J[k - 1] = jc;
        if ((k - 1) % 2 == 0) norm += (k == 1 ? 1.0 : 2.0) * jc;
        if (fabs(jc) > 1e200) {
          jc *= 1e-200;
          jp *= 1e-200;
          norm *= 1e-200;
          for (int i = k - 1; i <= K; ++i) J[i] *= 1e-200;
        }
      }
      const double inv = 1.0 / norm;
      for (int i = 0; i <= K; ++i) J[i] *= inv;
    }
    __syncthreads();
    const double inv_rho = 1.0 / rho;
    const double dx = (a - mu) * inv_rho, el = bl * inv_rho, er = br * inv_rho;
    auto xmul = [&](double w) {
      const double up = __shfl_up(w, 1, 64);    // row lane-1 (el = 0 on lane 0)
      const double dn = __shfl_down(w, 1, 64);  // row lane+1 (er = 0 on the last row)
      return dx * w + el * up + er * dn;
    };
    const double sg = (s > 0.0) ? 1.0 : -1.0;
    // (-i sg)^k: k % 4 = 0: 1, 1: -i sg, 2: -1, 3: +i sg
    auto acc = [&](int k, double w) {
      const double t = 2.0 * J[k] * w;
      switch (k & 3) {
        case 0: cr += t; break;
        case 1: ci -= sg * t; break;
        case 2: cr -= t; break;
        default: ci += sg * t; break;
      }
    };
    double w0 = (lane == 0) ? 1.0 : 0.0;
    cr = J[0] * w0;
    double w1 = xmul(w0);
    acc(1, w1);
    for (int k = 2; k <= K; ++k) {
      const double w2 = 2.0 * xmul(w1) - w0;
      acc(k, w2);
      w0 = w1;
      w1 = w2;
    }
  }
  const double ph = -tau * mu;
  const double pr = cos(ph), pi = sin(ph);
  const double fr = cr * pr - ci * pi, fi = cr * pi + ci * pr;
  if (act) {
    c_re[lane] = fr;
    c_im[lane] = fi;
    if (lane == m - 1) err[0] = beta[m - 1] * hypot(fr, fi);
  }
}

hipError_t launch_tridiag_expm(const double* alpha, const double* beta, int m, double tau,
                               double* c_re, double* c_im, double* err, hipStream_t s) {
  if (m < 1 || m > MAXV) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_expm_kernel, dim3(1), dim3(64), 0, s, alpha, beta, m, tau, c_re, c_im,
                     err, (const int*)nullptr);
  return hipGetLastError();
}

hipError_t launch_tridiag_expm_dev(const double* alpha, const double* beta, const int* jd, double tau,
                                   double* c_re, double* c_im, double* err, hipStream_t s) {
  hipLaunchKernelGGL(tridiag_expm_kernel, dim3(1), dim3(64), 0, s, alpha, beta, 1, tau, c_re, c_im, err, jd);
  return hipGetLastError();
}

// --------------------------------------------------------------- SVD bits ---
__global__ __launch_bounds__(256) void interleave_kernel(const double* planar, long n, double* z) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    z[2 * i] = planar[i];
    z[2 * i + 1] = planar[n + i];
  }
}

hipError_t launch_interleave(const double* planar, long n, double* z, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(interleave_kernel, stream_grid(n), dim3(256), 0, s, planar, n, z);
  return hipGetLastError();
}

// Single thread: sequential tail sums in ascending magnitude order.
__global__ void choose_rank_kernel(const double* S, int nsv, double eps, int D_max, int sv_mode,
                                   double tie_rel, int* out_k, double* out_disc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int k;
  if (sv_mode == 2) {
    k = nsv;
  } else if (sv_mode == 1) {
    k = 0;
    for (int j = 0; j < nsv; ++j)
      if (S[j] >= eps * S[0]) ++k;
  } else {
    double total = 0.0;
    for (int j = nsv - 1; j >= 0; --j) total += S[j] * S[j];
    // tail(j) = sum_{l >= j} s_l^2, accumulated from the smallest value;
    // k = smallest j >= 1 with tail(j) <= eps * total
    k = nsv;
    double tail = 0.0;
    for (int j = nsv - 1; j >= 1; --j) {
      tail += S[j] * S[j];
      if (tail <= eps * total) k = j;
      else break;
    }
  }
  if (k > D_max) k = D_max;
  if (k > nsv) k = nsv;
  if (k < 1) k = 1;
  if (sv_mode != 2) {
    const int lim = nsv < D_max ? nsv : D_max;
    while (k < lim && S[k] > 0.0 && S[k] >= (1.0 - tie_rel) * S[k - 1]) ++k;
  }
  double disc = 0.0;
  for (int j = nsv - 1; j >= k; --j) disc += S[j] * S[j];
  out_k[0] = k;
  out_disc[0] = disc;
}

hipError_t launch_choose_rank(const double* S, int nsv, double eps, int D_max, int sv_mode,
                              double tie_rel, int* out_k, double* out_disc, hipStream_t s) {
  hipLaunchKernelGGL(choose_rank_kernel, dim3(1), dim3(64), 0, s, S, nsv, eps, D_max, sv_mode,
                     tie_rel, out_k, out_disc);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void eig_to_sv_kernel(const double* lam, int n, double* S) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double v = lam[n - 1 - j];
    S[j] = v > 0.0 ? sqrt(v) : 0.0;
  }
}

hipError_t launch_eig_to_sv(const double* lam, int n, double* S, hipStream_t s) {
  hipLaunchKernelGGL(eig_to_sv_kernel, stream_grid(n), dim3(256), 0, s, lam, n, S);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void eigvec_extract_kernel(const double* Z, int n, int k, int conj,
                                                             int transpose, double* out) {
  const long tot = (long)n * k;
  const double sg = conj ? -1.0 : 1.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long)gridDim.x * blockDim.x) {
    int i, j;
    if (transpose) {  // out[j][i], i fastest (coalesced reads of a column of Z)
      j = (int)(t / n);
      i = (int)(t % n);
    } else {  // out[i][j]
      i = (int)(t / k);
      j = (int)(t % k);
    }
    const long src = 2 * ((long)i + (long)(n - 1 - j) * n);
    out[t] = Z[src];
    out[tot + t] = sg * Z[src + 1];
  }
}

hipError_t launch_eigvec_extract(const double* Z, int n, int k, int conj, int transpose,
                                 double* out, hipStream_t s) {
  hipLaunchKernelGGL(eigvec_extract_kernel, stream_grid((long)n * k), dim3(256), 0, s, Z, n, k, conj,
                     transpose, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_sv_kernel(double* m, int rows, int cols, const double* S,
                                                       int by_rows, int inv) {
  const long tot = (long)rows * cols;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long)gridDim.x * blockDim.x) {
    const int j = by_rows ? (int)(t / cols) : (int)(t % cols);
    const double s = S[j];
    const double f = inv ? (s > 0.0 ? 1.0 / s : 0.0) : s;
    m[t] *= f;
    m[tot + t] *= f;
  }
}

hipError_t launch_scale_sv(double* m, int rows, int cols, const double* S, int by_rows, int inv,
                           hipStream_t s) {
  hipLaunchKernelGGL(scale_sv_kernel, stream_grid((long)rows * cols), dim3(256), 0, s, m, rows, cols, S,
                     by_rows, inv);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_kernel(double* p, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(double* p, long n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, stream_grid(n), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void conj_transpose_kernel(const double* in, int nb, int n, double* out) {
  const long nn = (long)n * n, tot = (long)nb * nn;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long)gridDim.x * blockDim.x) {
    const long b = t / nn, r = t % nn;
    const int i = (int)(r / n), j = (int)(r % n);
    const long src = b * nn + (long)j * n + i;
    out[t] = in[src];
    out[tot + t] = -in[tot + src];
  }
}

hipError_t launch_conj_transpose(const double* in, int nb, int n, double* out, hipStream_t s) {
  const long tot = (long)nb * n * n;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(conj_transpose_kernel, stream_grid(tot), dim3(256), 0, s, in, nb, n, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void cscale_kernel(double* x, long n, double re, double im) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double a = x[i], b = x[n + i];
    x[i] = re * a - im * b;
    x[n + i] = re * b + im * a;
  }
}

hipError_t launch_cscale(double* x, long n, double re, double im, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cscale_kernel, stream_grid(n), dim3(256), 0, s, x, n, re, im);
  return hipGetLastError();
}

// ---------------------------------------------------- one-sided Jacobi SVD --
constexpr int JAC_THREADS = 1024;
constexpr int JAC_WAVES = JAC_THREADS / 64;

// Rotate the pair (x, y) of complex vectors (planar, stride-1, length len)
// with the G lanes of one pair slot:
// x' = c x - s e y,  y' = s x + c e y,  e = exp(-i phase).
template <int G>
__device__ __forceinline__ void jac_rotate(double* xr, double* xi, double* yr, double* yi, long stride,
                                           int len, int lane, double c, double s, double er, double ei) {
  for (int i = lane; i < len; i += G) {
    const long o = (long)i * stride;
    const double ar = xr[o], ai = xi[o], br = yr[o], bi = yi[o];
    const double eyr = er * br - ei * bi, eyi = er * bi + ei * br;
    xr[o] = c * ar - s * eyr;
    xi[o] = c * ai - s * eyi;
    yr[o] = s * ar + c * eyr;
    yi[o] = s * ai + c * eyi;
  }
}

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// G lanes per pair (64 or 16): with short vectors, four pairs per wave keep
// the workgroup's waves busy in each round.
template <int G>
__global__ __launch_bounds__(JAC_THREADS) void jacobi_svd_kernel(const double* theta, int rows, int cols,
                                                                 int left, double* W, double* V,
                                                                 double* sig, int* perm, int max_sweeps) {
  const int nv = left ? rows : cols;
  const int len = left ? cols : rows;
  const long wsz = (long)nv * len;
  const long vsz = (long)nv * nv;
  const long tsz = (long)rows * cols;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double fro = 0.0;
  for (long t = tid; t < wsz; t += JAC_THREADS) {
    const int j = (int)(t / len), i = (int)(t % len);
    const long src = left ? (long)j * cols + i : (long)i * cols + j;  // w_j[i]
    const double xr = theta[src], xi = theta[tsz + src];
    W[t] = xr;
    W[wsz + t] = (left ? -1.0 : 1.0) * xi;
    fro += xr * xr + xi * xi;
  }
  for (long t = tid; t < vsz; t += JAC_THREADS) {
    V[t] = ((t / nv) == (t % nv)) ? 1.0 : 0.0;
    V[vsz + t] = 0.0;
  }
  __shared__ int s_rot;
  __shared__ double s_sig[kJacobiMaxVectors];
  __shared__ double s_fro[JAC_WAVES];
  fro = wave_sum(fro);
  if (lane == 0) s_fro[wave] = fro;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < JAC_WAVES; ++w) fro2 += s_fro[w];
  // pairs whose norms are at rounding level of the whole matrix are left alone
  const double noise = 1e-28 * fro2;
  const int nvp = nv + (nv & 1);
  for (int sweep = 0; sweep < max_sweeps && nvp > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    const int slot = tid / G, glane = tid % G;
    for (int r = 0; r < nvp - 1; ++r) {
      // circle method: position 0 fixed, the others rotate by r
      for (int k = slot; k < nvp / 2; k += JAC_THREADS / G) {
        const int ia = k, ib = nvp - 1 - k;
        int p = ia == 0 ? 0 : ((ia - 1 + r) % (nvp - 1)) + 1;
        int q = ((ib - 1 + r) % (nvp - 1)) + 1;
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        if (q >= nv) continue;  // pairs with the padding index
        double* xr = W + (long)p * len;
        double* yr = W + (long)q * len;
        double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
        for (int i = glane; i < len; i += G) {
          const double ar = xr[i], ai = xr[wsz + i], br = yr[i], bi = yr[wsz + i];
          a += ar * ar + ai * ai;
          b += br * br + bi * bi;
          gr += ar * br + ai * bi;  // Re conj(x) y
          gi += ar * bi - ai * br;  // Im conj(x) y
        }
        a = group_sum<G>(a);
        b = group_sum<G>(b);
        gr = group_sum<G>(gr);
        gi = group_sum<G>(gi);
        const double g = hypot(gr, gi);
        const double ab = sqrt(a * b);
        if (g > 1e-15 * ab && ab > noise) {
          const double zeta = (b - a) / (2.0 * g);
          const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tn * tn), sn = c * tn;
          const double er = gr / g, ei = -gi / g;  // exp(-i phase of x^H y)
          jac_rotate<G>(xr, xr + wsz, yr, yr + wsz, 1, len, glane, c, sn, er, ei);
          // V is kept transposed (row j = column j of the accumulated
          // rotation), so both rotations stream contiguous memory
          jac_rotate<G>(V + (long)p * nv, V + vsz + (long)p * nv, V + (long)q * nv, V + vsz + (long)q * nv, 1, nv,
                        glane, c, sn, er, ei);
          if (glane == 0) s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int done = (s_rot == 0);
    __syncthreads();
    if (done) break;
  }
  for (int j = wave; j < nv; j += JAC_WAVES) {
    const double* x = W + (long)j * len;
    double a = 0.0;
    for (int i = lane; i < len; i += 64) a += x[i] * x[i] + x[wsz + i] * x[wsz + i];
    a = wave_sum(a);
    if (lane == 0) s_sig[j] = sqrt(a);
  }
  __syncthreads();
  for (int j = tid; j < nv; j += JAC_THREADS) {
    const double sj = s_sig[j];
    int rank = 0;
    for (int i = 0; i < nv; ++i)
      if (s_sig[i] > sj || (s_sig[i] == sj && i < j)) ++rank;
    sig[rank] = sj;
    perm[rank] = j;
  }
}

hipError_t launch_jacobi_svd(const double* theta, int rows, int cols, int left, double* Wk,
                             double* Vacc, double* sig, int* perm, int max_sweeps, hipStream_t s) {
  const int nv = left ? rows : cols;
  if (nv < 1 || nv > kJacobiMaxVectors) return hipErrorInvalidValue;
  const int len = left ? cols : rows;
  if (len <= 256 && nv >= 64)  // short vectors, enough pairs: four pairs per wave
    hipLaunchKernelGGL(jacobi_svd_kernel<16>, dim3(1), dim3(JAC_THREADS), 0, s, theta, rows, cols, left, Wk,
                       Vacc, sig, perm, max_sweeps);
  else
    hipLaunchKernelGGL(jacobi_svd_kernel<64>, dim3(1), dim3(JAC_THREADS), 0, s, theta, rows, cols, left, Wk,
                       Vacc, sig, perm, max_sweeps);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void jacobi_assemble_kernel(const double* W, const double* V,
                                                              const double* sig, const int* perm,
                                                              int rows, int cols, int left, int k,
                                                              int mode, double* out1, double* out2) {
  const int nv = left ? rows : cols;
  const int len = left ? cols : rows;
  const long wsz = (long)nv * len, vsz = (long)nv * nv;
  const long n1 = (long)rows * k, n2 = (long)k * cols;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n1 + n2; t += (long)gridDim.x * blockDim.x) {
    if (t < n1) {  // out1[r][jj]
      const int r = (int)(t / k), jj = (int)(t % k);
      const int j = perm[jj];
      if (left) {  // U = Vacc (stored transposed)
        out1[t] = V[(long)j * nv + r];
        out1[n1 + t] = V[vsz + (long)j * nv + r];
      } else {  // U S = W (columns); mode 0/1: U = W S^-1
        double f = 1.0;
        if (mode != 2) f = sig[jj] > 0.0 ? 1.0 / sig[jj] : 0.0;
        out1[t] = f * W[(long)j * len + r];
        out1[n1 + t] = f * W[wsz + (long)j * len + r];
      }
    } else {  // out2[jj][c]
      const long u = t - n1;
      const int jj = (int)(u / cols), c = (int)(u % cols);
      const int j = perm[jj];
      if (left) {  // S Vh = W^H, optionally divided by S
        double f = 1.0;
        if (mode == 0) f = sig[jj] > 0.0 ? 1.0 / sig[jj] : 0.0;
        out2[u] = f * W[(long)j * len + c];
        out2[n2 + u] = -f * W[wsz + (long)j * len + c];
      } else {  // Vh = Vacc^H (Vacc stored transposed)
        out2[u] = V[(long)j * nv + c];
        out2[n2 + u] = -V[vsz + (long)j * nv + c];
      }
    }
  }
}

hipError_t launch_jacobi_assemble(const double* Wk, const double* Vacc, const double* sig,
                                  const int* perm, int rows, int cols, int left, int k, int mode,
                                  double* out1, double* out2, hipStream_t s) {
  const long tot = (long)rows * k + (long)k * cols;
  hipLaunchKernelGGL(jacobi_assemble_kernel, stream_grid(tot), dim3(256), 0, s, Wk, Vacc, sig, perm, rows,
                     cols, left, k, mode, out1, out2);
  return hipGetLastError();
}

// ------------------------------------------------------------- adjoints ---
// Z[j][i] /= (s_keep[i]^2 - s_perp[j]^2) for a planar kp x k matrix; pairs
// closer than 1e-14 s_all[0]^2 are zeroed.
__global__ __launch_bounds__(256) void gap_scale_kernel(double* Z, int kp, int k, const double* s_perp,
                                                        const double* s_keep, const double* s_all) {
  const long n = (long)kp * k;
  const double s0 = s_all[0];
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / k), i = (int)(t % k);
    const double den = s_keep[i] * s_keep[i] - s_perp[j] * s_perp[j];
    const double f = fabs(den) > 1e-14 * s0 * s0 ? 1.0 / den : 0.0;
    Z[t] *= f;
    Z[n + t] *= f;
  }
}

hipError_t launch_gap_scale(double* Z, int kp, int k, const double* s_perp, const double* s_keep, const double* s_all,
                            hipStream_t s) {
  if ((long)kp * k == 0) return hipSuccess;
  hipLaunchKernelGGL(gap_scale_kernel, stream_grid((long)kp * k), dim3(256), 0, s, Z, kp, k, s_perp, s_keep, s_all);
  return hipGetLastError();
}

// X[i][j] /= S[j]^2 (zero when S[j] == 0) for a planar rows x cols matrix.
__global__ __launch_bounds__(256) void scale_cols_inv2_kernel(double* X, int rows, int cols, const double* S) {
  const long n = (long)rows * cols;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const double v = S[t % cols];
    const double f = v > 0.0 ? 1.0 / (v * v) : 0.0;
    X[t] *= f;
    X[n + t] *= f;
  }
}

hipError_t launch_scale_cols_inv2(double* X, int rows, int cols, const double* S, hipStream_t s) {
  hipLaunchKernelGGL(scale_cols_inv2_kernel, stream_grid((long)rows * cols), dim3(256), 0, s, X, rows, cols, S);
  return hipGetLastError();
}

// out[j][i] = conj(in[i][j]) for a planar rows x cols matrix (out: cols x rows).
__global__ __launch_bounds__(256) void conj_transpose_rect_kernel(const double* in, int rows, int cols, double* out) {
  const long n = (long)rows * cols;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const long j = t / rows, i = t % rows;  // coalesced reads of a column of in
    const long src = i * cols + j;
    out[t] = in[src];
    out[n + t] = -in[n + src];
  }
}

hipError_t launch_conj_transpose_rect(const double* in, int rows, int cols, double* out, hipStream_t s) {
  hipLaunchKernelGGL(conj_transpose_rect_kernel, stream_grid((long)rows * cols), dim3(256), 0, s, in, rows, cols, out);
  return hipGetLastError();
}

// ------------------------------------------------ subspace-iteration SVD ---
// Counter-based uniform numbers in [-1, 1): SplitMix64 (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", 2014) of seed + t * golden.
__global__ __launch_bounds__(256) void randfill_kernel(double* x, long n, unsigned long long seed) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    unsigned long long z = seed + (unsigned long long)t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[t] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

hipError_t launch_randfill(double* x, long n, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(randfill_kernel, stream_grid(n), dim3(256), 0, s, x, n, seed);
  return hipGetLastError();
}

// Columns j0 .. b-1 of a planar row-major p x b matrix, same generator.
__global__ __launch_bounds__(256) void randfill_cols_kernel(double* x, int p, int b, int j0, unsigned long long seed) {
  const int w = b - j0;
  const long n = (long)p * w;
  const long plane = (long)p * b;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < 2 * n; t += (long)gridDim.x * blockDim.x) {
    const long e = t % n;
    const long dst = (t / n) * plane + (e / w) * b + j0 + e % w;
    unsigned long long z = seed + (unsigned long long)t * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[dst] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

hipError_t launch_randfill_cols(double* x, int p, int b, int j0, unsigned long long seed, hipStream_t s) {
  if (j0 >= b) return hipSuccess;
  if (j0 < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(randfill_cols_kernel, stream_grid(2L * p * (b - j0)), dim3(256), 0, s, x, p, b, j0, seed);
  return hipGetLastError();
}

// Pieces of the blocked Cholesky factorisation with triangular inverse used
// by the Cholesky QR orthonormalisation (the recursion and its GEMMs are on
// the host side).
//
// Column scaling of a Gram matrix: d_i = 1 / sqrt(G_ii), G <- diag(d) G diag(d).
// status[0] = 1 when a diagonal entry is zero or not finite (only written on
// failure).  One workgroup.
constexpr int CHOL_THREADS = 1024;

__global__ __launch_bounds__(CHOL_THREADS) void gram_colscale_kernel(double* G, int b, double* d, int* status,
                                                                      double shift) {
  __shared__ double dsc[kMaxSubspace];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const long bb = (long)b * b;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int i = tid; i < b; i += CHOL_THREADS) {
    const double g = G[(long)i * b + i];
    const bool ok = g > 0.0 && g < INFINITY;
    dsc[i] = ok ? 1.0 / sqrt(g) : 0.0;
    d[i] = dsc[i];
    if (!ok) bad = 1;
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) status[0] = 1;
    return;
  }
  for (long e = tid; e < bb; e += CHOL_THREADS) {
    const long r = e / b, c = e % b;
    const double f = dsc[r] * dsc[c];
    G[e] = G[e] * f + (r == c ? shift : 0.0);
    G[bb + e] *= f;
  }
}

hipError_t launch_gram_colscale(double* G, int b, double* d, int* status, hipStream_t s, double shift) {
  if (b < 1 || b > kMaxSubspace) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gram_colscale_kernel, dim3(1), dim3(CHOL_THREADS), 0, s, G, b, d, status, shift);
  return hipGetLastError();
}

// Leaf of the recursion: for the n x n block A (upper triangle read; planar
// with imaginary plane at im_a, row stride lda) computes A = R^H R in LDS and
// writes Rinv = R^(-1) (upper triangular, zeros below) to the n x n block at
// Rinv (imaginary plane at im_r, row stride ldr).  n <= kCholLeaf.
// status[0] = 2 when A is not positive definite (only written on failure).
// Both phases are right-looking with two barriers per step and the trailing
// work spread over a 16 x 16 thread grid: the Cholesky update of the trailing
// triangle, then R^(-1) by back substitution in which finishing row k of
// R^(-1) immediately updates the pending sums of every row above it.
constexpr int LEAF_THREADS = 256;

__global__ __launch_bounds__(LEAF_THREADS) void chol_leaf_kernel(const double* A, long im_a, long lda, int n,
                                                                double* Rinv, long im_r, long ldr, int* status) {
  __shared__ double Rr[kCholLeaf][kCholLeaf + 1], Ri[kCholLeaf][kCholLeaf + 1];
  __shared__ double Tr[kCholLeaf][kCholLeaf + 1], Ti[kCholLeaf][kCholLeaf + 1];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int i = ty; i < n; i += 16)
    for (int j = tx; j < n; j += 16) {
      Rr[i][j] = j >= i ? A[(long)i * lda + j] : 0.0;
      Ri[i][j] = j > i ? A[im_a + (long)i * lda + j] : 0.0;
      Tr[i][j] = (i == j) ? 1.0 : 0.0;  // pending sums of the back substitution
      Ti[i][j] = 0.0;
    }
  __syncthreads();
  // A = R^H R: step k scales row k by 1/sqrt(pivot) and updates the trailing
  // triangle with the outer product of the scaled row.
  for (int k = 0; k < n; ++k) {
    const double piv = Rr[k][k];  // final since the previous step's barrier
    if (!(piv > 0.0)) {           // the same value in every thread: uniform exit
      if (tid == 0) status[0] = 2;
      return;
    }
    const double rinv = 1.0 / sqrt(piv);
    for (int j = k + 1 + tid; j < n; j += LEAF_THREADS) {
      Rr[k][j] *= rinv;
      Ri[k][j] *= rinv;
    }
    __syncthreads();
    for (int i = k + 1 + ty; i < n; i += 16) {
      const double fr = Rr[k][i], fi = -Ri[k][i];  // conj(R_ki)
      for (int j = k + 1 + tx; j < n; j += 16) {
        if (j < i) continue;
        const double br = Rr[k][j], bi = Ri[k][j];
        Rr[i][j] -= fr * br - fi * bi;
        Ri[i][j] -= fr * bi + fi * br;
      }
    }
    if (tid == 0) Rr[k][k] = piv * rinv;  // sqrt(piv); no thread reads it before the barrier
    __syncthreads();
  }
  // R T = I, rows from the bottom: T[k][.] = S[k][.] / R_kk, then S[i][.] -=
  // R_ik T[k][.] for every i < k (S starts as the identity, held in T).
  for (int k = n - 1; k >= 0; --k) {
    const double dinv = 1.0 / Rr[k][k];
    for (int j = k + tid; j < n; j += LEAF_THREADS) {
      Tr[k][j] *= dinv;
      Ti[k][j] *= dinv;
    }
    __syncthreads();
    for (int i = ty; i < k; i += 16) {
      const double fr = Rr[i][k], fi = Ri[i][k];
      for (int j = k + tx; j < n; j += 16) {
        const double br = Tr[k][j], bi = Ti[k][j];
        Tr[i][j] -= fr * br - fi * bi;
        Ti[i][j] -= fr * bi + fi * br;
      }
    }
    __syncthreads();
  }
  for (int i = ty; i < n; i += 16)
    for (int j = tx; j < n; j += 16) {
      Rinv[(long)i * ldr + j] = Tr[i][j];
      Rinv[im_r + (long)i * ldr + j] = Ti[i][j];
    }
}

hipError_t launch_chol_leaf(const double* A, long im_a, long lda, int n, double* Rinv, long im_r, long ldr,
                            int* status, hipStream_t s) {
  if (n < 1 || n > kCholLeaf) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_leaf_kernel, dim3(1), dim3(LEAF_THREADS), 0, s, A, im_a, lda, n, Rinv, im_r, ldr, status);
  return hipGetLastError();
}

// T[i][j] *= d[i] for a planar b x b matrix.
__global__ __launch_bounds__(256) void rowscale_kernel(double* T, int b, const double* d) {
  const long bb = (long)b * b;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < bb; e += (long)gridDim.x * blockDim.x) {
    const double f = d[e / b];
    T[e] *= f;
    T[bb + e] *= f;
  }
}

hipError_t launch_rowscale(double* T, int b, const double* d, hipStream_t s) {
  hipLaunchKernelGGL(rowscale_kernel, stream_grid((long)b * b), dim3(256), 0, s, T, b, d);
  return hipGetLastError();
}

// Column norms of a planar row-major matrix: partial sums over row chunks,
// then a fixed-order reduction of the chunks.
constexpr int CN_CHUNKS = 32;

__global__ __launch_bounds__(256) void colnorm_part_kernel(const double* P, long im, int rows, long ld,
                                                          int ncols, double* part) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + tx;
  const int chunk = blockIdx.y;
  const int per = (rows + CN_CHUNKS - 1) / CN_CHUNKS;
  const int r0 = chunk * per, r1 = min(rows, r0 + per);
  double acc = 0.0;
  if (c < ncols) {
    for (int i = r0 + ty; i < r1; i += 4) {
      const double re = P[(long)i * ld + c], iv = P[im + (long)i * ld + c];
      acc += re * re + iv * iv;
    }
  }
  red[ty][tx] = acc;
  __syncthreads();
  if (ty == 0 && c < ncols) part[(long)chunk * ncols + c] = red[0][tx] + red[1][tx] + red[2][tx] + red[3][tx];
}

__global__ __launch_bounds__(256) void colnorm_final_kernel(const double* part, int ncols, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double acc = 0.0;
  for (int k = 0; k < CN_CHUNKS; ++k) acc += part[(long)k * ncols + c];
  out[c] = sqrt(acc);
}

hipError_t launch_colnorms(const double* P, long im, int rows, long ld, int ncols, double* part, double* out,
                           hipStream_t s) {
  if (ncols < 1) return hipSuccess;
  hipLaunchKernelGGL(colnorm_part_kernel, dim3((ncols + 63) / 64, CN_CHUNKS), dim3(256), 0, s, P, im, rows, ld,
                     ncols, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colnorm_final_kernel, dim3((ncols + 255) / 256), dim3(256), 0, s, part, ncols, out);
  return hipGetLastError();
}

long colnorm_part_doubles(int ncols) { return (long)CN_CHUNKS * ncols; }

// Rank selection from the leading nb singular values and the Frobenius norm
// of the whole matrix (norm[0]): the tail weight beyond index j is
// norm^2 - sum_{l<j} S_l^2.  Same rule as choose_rank_kernel otherwise.
__global__ void choose_rank_partial_kernel(const double* S, int nb, const double* norm, double eps, int D_max,
                                           int sv_mode, double tie_rel, int* out_k, double* out_disc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double total = norm[0] * norm[0];
  int k;
  if (sv_mode == 1) {
    k = 0;
    for (int j = 0; j < nb; ++j)
      if (S[j] >= eps * S[0]) ++k;
  } else {
    k = nb;
    double kept = 0.0;
    for (int j = 1; j <= nb; ++j) {
      kept += S[j - 1] * S[j - 1];
      if (total - kept <= eps * total) {
        k = j;
        break;
      }
    }
  }
  if (k > D_max) k = D_max;
  if (k > nb) k = nb;
  if (k < 1) k = 1;
  const int lim = nb < D_max ? nb : D_max;
  while (k < lim && S[k] > 0.0 && S[k] >= (1.0 - tie_rel) * S[k - 1]) ++k;
  double kept = 0.0;
  for (int j = 0; j < k; ++j) kept += S[j] * S[j];
  const double disc = total - kept;
  out_k[0] = k;
  out_disc[0] = disc > 0.0 ? disc : 0.0;
}

hipError_t launch_choose_rank_partial(const double* S, int nb, const double* norm, double eps, int D_max,
                                      int sv_mode, double tie_rel, int* out_k, double* out_disc, hipStream_t s) {
  hipLaunchKernelGGL(choose_rank_partial_kernel, dim3(1), dim3(64), 0, s, S, nb, norm, eps, D_max, sv_mode,
                     tie_rel, out_k, out_disc);
  return hipGetLastError();
}

// sigma[m] = (1 / (pi hbar)) Re sum_k w_k C_k exp(i E_m t_k / hbar - t_k / tau)
// with t_k = k dt and trapezoid weights w_k (dt, halved at both ends): one
// thread per energy, the samples staged through LDS in chunks.
constexpr int SPEC_THREADS = 256;
constexpr int SPEC_CHUNK = 512;

__global__ __launch_bounds__(SPEC_THREADS) void spectrum_kernel(const double* C, int N, double dt, double inv_tau,
                                                                double hbar, const double* E, int M, double* sigma) {
  __shared__ double cr[SPEC_CHUNK], ci[SPEC_CHUNK];
  const int m = blockIdx.x * SPEC_THREADS + threadIdx.x;
  const double e = m < M ? E[m] / hbar : 0.0;
  double acc = 0.0;
  for (int k0 = 0; k0 < N; k0 += SPEC_CHUNK) {
    const int nk = min(SPEC_CHUNK, N - k0);
    __syncthreads();
    for (int j = threadIdx.x; j < nk; j += SPEC_THREADS) {
      const int k = k0 + j;
      const double wk = (k == 0 || k == N - 1) ? 0.5 * dt : dt;
      const double damp = wk * exp(-(k * dt) * inv_tau);
      cr[j] = C[k] * damp;
      ci[j] = C[N + k] * damp;
    }
    __syncthreads();
    if (m < M) {
      for (int j = 0; j < nk; ++j) {
        double sn, cs;
        sincos(e * ((k0 + j) * dt), &sn, &cs);
        acc += cr[j] * cs - ci[j] * sn;  // Re[(cr + i ci)(cs + i sn)]
      }
    }
  }
  if (m < M) sigma[m] = acc / (M_PI * hbar);
}

hipError_t launch_spectrum(const double* C, int N, double dt, double tau, double hbar, const double* E, int M,
                           double* sigma, hipStream_t s) {
  if (N < 1 || M < 1) return hipSuccess;
  hipLaunchKernelGGL(spectrum_kernel, dim3((M + SPEC_THREADS - 1) / SPEC_THREADS), dim3(SPEC_THREADS), 0, s, C, N,
                     dt, 1.0 / tau, hbar, E, M, sigma);
  return hipGetLastError();
}


// ------------------------------------------------ whole-MPS building blocks --
// MPO x MPS on one site: out[(a wl + w)][s][(b wr + y)] = sum_t W[w][y][s][t]
// A[a][t][b], planar (W [2][wl][wr][d][d], A [2][Dl][d][Dr]); one output
// element per thread, the t sum in order.
__global__ __launch_bounds__(256) void mpo_apply_kernel(const double* __restrict__ W, int wl, int wr, int d,
                                                        const double* __restrict__ A, int Dl, int Dr,
                                                        double* __restrict__ out) {
  const long DR = (long)Dr * wr;
  const long total = (long)Dl * wl * d * DR;
  const long wim = (long)wl * wr * d * d, aim = (long)Dl * d * Dr;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long col = idx % DR, rest = idx / DR;
    const int s = (int)(rest % d);
    const long row = rest / d;
    const int a = (int)(row / wl), w = (int)(row % wl);
    const int b = (int)(col / wr), y = (int)(col % wr);
    const double* wp = W + (((long)w * wr + y) * d + s) * d;
    const double* ap = A + (long)a * d * Dr + b;
    double re = 0.0, im = 0.0;
    for (int t = 0; t < d; ++t) {
      const double xr = wp[t], xi = wp[wim + t];
      const double yr = ap[(long)t * Dr], yi = ap[aim + (long)t * Dr];
      re += xr * yr - xi * yi;
      im += xr * yi + xi * yr;
    }
    out[idx] = re;
    out[total + idx] = im;
  }
}

hipError_t launch_mpo_apply(const double* W, int wl, int wr, int d, const double* A, int Dl, int Dr, double* out,
                            hipStream_t s) {
  const long total = (long)Dl * wl * d * Dr * wr;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(mpo_apply_kernel, stream_grid(total), dim3(256), 0, s, W, wl, wr, d, A, Dl, Dr, out);
  return hipGetLastError();
}

// dst[a0 + a][s][b0 + b] = c src[a][s][b] (dst [2][Ld][d][Rd], src [2][Ls][d][Rs]).
__global__ __launch_bounds__(256) void block_copy_kernel(double* __restrict__ dst, int Ld, int Rd,
                                                         const double* __restrict__ src, int Ls, int Rs, int d,
                                                         int a0, int b0, double cr, double ci) {
  const long total = (long)Ls * d * Rs;
  const long dim = (long)Ld * d * Rd;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int b = (int)(idx % Rs);
    const long rest = idx / Rs;
    const int sd = (int)(rest % d), a = (int)(rest / d);
    const long o = ((long)(a0 + a) * d + sd) * Rd + b0 + b;
    const double xr = src[idx], xi = src[total + idx];
    dst[o] = cr * xr - ci * xi;
    dst[dim + o] = cr * xi + ci * xr;
  }
}

hipError_t launch_block_copy(double* dst, int Ld, int Rd, const double* src, int Ls, int Rs, int d, int a0, int b0,
                             double cr, double ci, hipStream_t s) {
  const long total = (long)Ls * d * Rs;
  if (total <= 0) return hipSuccess;
  if (a0 < 0 || b0 < 0 || a0 + Ls > Ld || b0 + Rs > Rd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_copy_kernel, stream_grid(total), dim3(256), 0, s, dst, Ld, Rd, src, Ls, Rs, d, a0, b0,
                     cr, ci);
  return hipGetLastError();
}


// out[j][i][e] (+)= in[i][j][e]: the two outer axes of a planar complex array
// exchanged; index order of out, so reads and writes both run along e.
__global__ __launch_bounds__(256) void swap_outer_kernel(const double* __restrict__ in, long in_im, int n1, int n2,
                                                         long q, double* __restrict__ out, long out_im, int acc) {
  const long total = (long)n1 * n2 * q;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long e = idx % q;
    const long t = idx / q;
    const long i = t % n1, j = t / n1;
    const long src = (i * n2 + j) * q + e;
    double xr = in[src], xi = in[in_im + src];
    if (acc) {
      xr += out[idx];
      xi += out[out_im + idx];
    }
    out[idx] = xr;
    out[out_im + idx] = xi;
  }
}

hipError_t launch_swap_outer(const double* in, long in_im, int n1, int n2, long q, double* out, long out_im,
                             bool acc, hipStream_t s) {
  const long total = (long)n1 * n2 * q;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(swap_outer_kernel, stream_grid(total), dim3(256), 0, s, in, in_im, n1, n2, q, out, out_im,
                     acc ? 1 : 0);
  return hipGetLastError();
}

// out[i][j] = A[i * ld + j] (interleaved complex A, planar out [2][nrow][ncol])
// for i < nrow, j < ncol, with mask 1 keeping j >= i, 2 keeping j <= i (zero
// elsewhere), 0 everything.
__global__ __launch_bounds__(256) void extract_ld_kernel(const double* __restrict__ A, long ld, int nrow, int ncol,
                                                         int mask, double* __restrict__ out) {
  const long total = (long)nrow * ncol;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / ncol), j = (int)(idx % ncol);
    const bool keep = mask == 0 || (mask == 1 && j >= i) || (mask == 2 && j <= i);
    const long a = 2 * ((long)i * ld + j);
    out[idx] = keep ? A[a] : 0.0;
    out[total + idx] = keep ? A[a + 1] : 0.0;
  }
}

hipError_t launch_extract_ld(const double* A, long ld, int nrow, int ncol, int mask, double* out, hipStream_t s) {
  const long total = (long)nrow * ncol;
  if (total <= 0) return hipSuccess;
  if (ncol > ld) return hipErrorInvalidValue;
  hipLaunchKernelGGL(extract_ld_kernel, stream_grid(total), dim3(256), 0, s, A, ld, nrow, ncol, mask, out);
  return hipGetLastError();
}

}  // namespace tdmrg
