// Block-Jacobi preconditioned CG over s right-hand sides in lock-step
// (Algorithm 2, the two solves), from x0 = 0.
//
// Every per-column scalar (rho, alpha, beta, the residual test) lives on the
// device and is produced by one-block kernels from partial sums written in a
// fixed order, so the loop needs no host round trip per iteration: the host
// only reads the status every few iterations.  Once all columns have met the
// tolerance (or an error stopped the loop) every kernel of the loop returns at
// once, so iterations queued past convergence cost a launch each.
//
// Column j freezes (x_j, r_j, p_j no longer change) when
// ||r_j|| <= tol ||b_j|| on the recurrence residual.
#include <algorithm>
#include <chrono>
#include <climits>

#include "common.h"

namespace firal {

// part[j * P + p] = sum over a in slice p of sum_k A[a,j,k] B[a,j,k].
template <typename T>
__global__ __launch_bounds__(256) void k_coldot(const T* __restrict__ A, const T* __restrict__ B,
                                                int d, int s, int c, int P,
                                                double* __restrict__ part, Skip skip) {
  if (skip_now(skip)) return;
  const int j = blockIdx.x, p = blockIdx.y;
  const int per = (d + P - 1) / P;
  const int a0 = p * per;
  const int a1 = min(d, a0 + per);
  const int64_t n = a1 > a0 ? (int64_t)(a1 - a0) * c : 0;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int a = a0 + (int)(e / c), k = (int)(e % c);
    const int64_t i = ((int64_t)a * s + j) * c + k;
    acc += (double)A[i] * (double)B[i];
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) part[j * P + p] = acc;
}

int coldot_launch(Ctx* x, const void* A, const void* B, int s, double* part, Skip skip,
                  hipStream_t st) {
  dim3 grid(s, x->col_parts);
  if (x->prec == FIRAL_F64)
    k_coldot<double><<<grid, 256, 0, st>>>((const double*)A, (const double*)B, x->d, s, x->c,
                                           x->col_parts, part, skip);
  else
    k_coldot<float><<<grid, 256, 0, st>>>((const float*)A, (const float*)B, x->d, s, x->c,
                                          x->col_parts, part, skip);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// Y[a,j,:] = R[a,j,:] - mean_k R[a,j,k]  (projection onto the complement of 1_c (x) u).
// Y may alias R.  One wave per (a, j) row of c classes: the lanes read the row coalesced,
// sum in FP64 (lane partials in class order, then the fixed-order wave sum), and write the
// row after every lane's reads of it have entered the sum.
constexpr int kRowWaves = 4;   // rows per 256-thread block
template <typename T>
__device__ __forceinline__ double row_mean(const T* r, int c, int lane) {
  double m = 0.0;
  for (int k = lane; k < c; k += 64) m += (double)r[k];
  return wave_sum(m) / c;
}
template <typename T>
__global__ __launch_bounds__(256) void k_project(const T* R, T* Y, int d, int s, int c,
                                                 Skip skip) {
  if (skip_now(skip)) return;
  const int64_t row = (int64_t)blockIdx.x * kRowWaves + (threadIdx.x >> 6);
  if (row >= (int64_t)d * s) return;
  const int lane = threadIdx.x & 63;
  const T* r = R + row * c;
  T* y = Y + row * c;
  const double m = row_mean(r, c, lane);
  for (int k = lane; k < c; k += 64) y[k] = (T)((double)r[k] - m);
}

// mean[a*s + j] = mean_k R[a,j,k] (one wave per row, as above)
template <typename T>
__global__ __launch_bounds__(256) void k_classmean(const T* __restrict__ R, double* __restrict__ mean,
                                                   int d, int s, int c, Skip skip) {
  if (skip_now(skip)) return;
  const int64_t row = (int64_t)blockIdx.x * kRowWaves + (threadIdx.x >> 6);
  if (row >= (int64_t)d * s) return;
  const int lane = threadIdx.x & 63;
  const double m = row_mean(R + row * c, c, lane);
  if (lane == 0) mean[row] = m;
}

// Z[a,j,k] = sum_b Pinv_k[b][a] (R[b,j,k] - mean[b,j]) for the probes j0 .. j0 + jn - 1
// (jn <= JT) of one class k per block (PROJ: the class means given).  The group's right-hand
// sides are staged in LDS as [b][j] (read as 16-byte broadcasts; rows padded with zeros to a
// multiple of 8); each thread takes rows a = tid, tid + 256, ... and streams column a of Pinv_k
// (P_k is symmetric) in batches of 8 rows b, the next batch loaded while the current one is
// used, consecutive threads reading consecutive addresses, so a group reads each block once:
// with up to 16 probes in one group (d <= 512), Pinv is read once per apply.  Each XCD takes a
// contiguous range of blocks (classes), so the classes that share a cache line of R and Z (class
// is their innermost index) meet in one L2.  Each output is one sequential sum over b.
constexpr int kApplyB = 8;   // rows b per batch
template <int JT> inline size_t papply_lds(int d) {
  return (size_t)cdiv(d, kApplyB) * kApplyB * JT * sizeof(double);
}
template <typename T, int JT, bool PROJ>
__global__ __launch_bounds__(256) void k_papply(const double* __restrict__ Pinv,
                                                const T* __restrict__ R,
                                                const double* __restrict__ mean,
                                                T* __restrict__ Z, int d, int s, int c,
                                                Skip skip) {
  static_assert(JT % 2 == 0, "right-hand sides read in pairs");
  if (skip_now(skip)) return;
  extern __shared__ __align__(16) double rs[];   // [dp][JT]
  const int64_t nb = gridDim.x, q = nb >> 3, rm = nb & 7;
  const int64_t x = blockIdx.x & 7, lid = x * q + (x < rm ? x : rm) + (blockIdx.x >> 3);
  const int ng = (s + JT - 1) / JT;
  const int k = (int)(lid / ng);
  const int j0 = (int)(lid - (int64_t)k * ng) * JT;
  const int jn = min(JT, s - j0);
  const int64_t sc = (int64_t)s * c;
  const int dp = (d + kApplyB - 1) / kApplyB * kApplyB;
  // staging in batches of 8 elements per thread: the 8 loads (clamped addresses) are issued
  // together, then the 8 LDS stores
  for (int e0 = 0; e0 < dp * JT; e0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + (int)threadIdx.x + 256 * u, b = e / JT, jj = e - b * JT;
      const bool ok = jj < jn && b < d;
      const int bc = ok ? b : 0, jc = ok ? jj : 0;
      v[u] = (double)R[bc * sc + (int64_t)(j0 + jc) * c + k];
      if constexpr (PROJ) v[u] -= mean[(int64_t)bc * s + j0 + jc];
      v[u] = ok ? v[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + (int)threadIdx.x + 256 * u;
      if (e < dp * JT) rs[e] = v[u];
    }
  }
  __syncthreads();
  const double* Pk = Pinv + (int64_t)k * d * d;
  for (int a = threadIdx.x; a < d; a += blockDim.x) {
    double acc[JT];
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) acc[jj] = 0.0;
    // rows b >= d of a batch read row d - 1 and are weighted by the zero pad of rs
    auto fetch = [&](int b0, double (&p)[kApplyB]) {
#pragma unroll
      for (int u = 0; u < kApplyB; ++u) {
        const int b = b0 + u < d ? b0 + u : d - 1;
        p[u] = Pk[(int64_t)b * d + a];
      }
    };
    double pc[kApplyB], pn[kApplyB];
    fetch(0, pc);
    for (int b0 = 0; b0 < dp; b0 += kApplyB) {
      fetch(b0 + kApplyB < dp ? b0 + kApplyB : b0, pn);
#pragma unroll
      for (int u = 0; u < kApplyB; ++u) {
        const double* r = rs + (b0 + u) * JT;
#pragma unroll
        for (int jj = 0; jj < JT; jj += 2) {
          const double2 rv = *reinterpret_cast<const double2*>(r + jj);
          acc[jj] = fma(pc[u], rv.x, acc[jj]);
          acc[jj + 1] = fma(pc[u], rv.y, acc[jj + 1]);
        }
      }
#pragma unroll
      for (int u = 0; u < kApplyB; ++u) pc[u] = pn[u];
    }
#pragma unroll
    for (int jj = 0; jj < JT; ++jj)
      if (jj < jn) Z[a * sc + (int64_t)(j0 + jj) * c + k] = (T)acc[jj];
  }
}

template <typename T, int JT>
static void papply_launch(const double* Pinv, const T* r, const double* mean, T* z, int d, int s,
                          int c, Skip skip, hipStream_t st) {
  const dim3 grid((unsigned)(c * cdiv(s, JT)));
  if (mean)
    k_papply<T, JT, true><<<grid, 256, papply_lds<JT>(d), st>>>(Pinv, r, mean, z, d, s, c, skip);
  else
    k_papply<T, JT, false><<<grid, 256, papply_lds<JT>(d), st>>>(Pinv, r, mean, z, d, s, c, skip);
}

// ------------------------------------------------------------ scalars

__device__ __forceinline__ double sum_parts(const double* part, int j, int P) {
  // independent loads first, then the fixed-order sum
  double v[64];
  const int m = P < 64 ? P : 64;
  for (int p = 0; p < m; ++p) v[p] = part[j * P + p];
  double acc = 0.0;
  for (int p = 0; p < m; ++p) acc += v[p];
  for (int p = m; p < P; ++p) acc += part[j * P + p];
  return acc;
}

__global__ __launch_bounds__(64) void k_cg_init(const double* part_bb, const double* part_rz, int s,
                                                int P, Status* st, double* rho, double* bnorm,
                                                double* relres, int32_t* done) {
  __shared__ int alldone;
  if (threadIdx.x == 0) alldone = 1;
  __syncthreads();
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    const double bb = sum_parts(part_bb, j, P);
    bnorm[j] = sqrt(bb);
    rho[j] = sum_parts(part_rz, j, P);
    done[j] = bb == 0.0;
    relres[j] = bb > 0.0 ? 1.0 : 0.0;
    if (bb != 0.0) atomicAnd(&alldone, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->iters = 0;
    // an earlier failure (non-SPD block, breakdown in a previous solve) stops this one too
    st->all_done = alldone || st->breakdown != 0 || st->bad_block != INT_MAX;
    double m = 0.0;
    for (int j = 0; j < s; ++j) m = fmax(m, relres[j]);
    st->relres_max = m;
  }
}

__global__ __launch_bounds__(64) void k_cg_alpha(const double* part_pq, int s, int P, Status* st,
                                                 const double* rho, const int32_t* done,
                                                 double* alpha) {
  if (st->all_done) return;
  __shared__ int brk;
  if (threadIdx.x == 0) brk = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    const double pq = sum_parts(part_pq, j, P);
    double a = 0.0;
    if (!done[j]) {
      if (!(pq > 0.0)) atomicOr(&brk, 1);
      else a = rho[j] / pq;
    }
    alpha[j] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0 && brk) {
    st->breakdown = 1;
    st->all_done = 1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_update(T* __restrict__ xv, T* __restrict__ r,
                                                   const T* __restrict__ p,
                                                   const T* __restrict__ q,
                                                   const double* __restrict__ alpha, int64_t n,
                                                   int s, int c, Skip skip) {
  if (skip_now(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = (int)((i / c) % s);
  const T a = (T)alpha[j];
  xv[i] += a * p[i];
  r[i] -= a * q[i];
}

__global__ __launch_bounds__(64) void k_cg_done(const double* part_rr, int s, int P, Status* st,
                                                const double* bnorm, double* relres,
                                                int32_t* done, double tol) {
  if (st->all_done) return;
  __shared__ int alldone;
  if (threadIdx.x == 0) alldone = 1;
  __syncthreads();
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    const double rn = sqrt(sum_parts(part_rr, j, P));
    if (!done[j] && rn <= tol * bnorm[j]) done[j] = 1;
    relres[j] = bnorm[j] > 0.0 ? rn / bnorm[j] : 0.0;
    if (!done[j]) atomicAnd(&alldone, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->iters += 1;
    double m = 0.0;
    for (int j = 0; j < s; ++j) m = fmax(m, relres[j]);
    st->relres_max = m;
    st->all_done = alldone;
  }
}

__global__ __launch_bounds__(64) void k_cg_beta(const double* part_rz, int s, int P, Status* st,
                                                double* rho, const int32_t* done, double* beta) {
  if (st->all_done) return;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    const double rz = sum_parts(part_rz, j, P);
    if (!done[j]) {
      beta[j] = rz / (rho[j] != 0.0 ? rho[j] : 1.0);
      rho[j] = rz;
    } else {
      beta[j] = 0.0;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_pupdate(T* __restrict__ p, const T* __restrict__ z,
                                                    const double* __restrict__ beta,
                                                    const int32_t* __restrict__ done, int64_t n,
                                                    int s, int c, Skip skip) {
  if (skip_now(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = (int)((i / c) % s);
  if (done[j]) return;
  p[i] = z[i] + (T)beta[j] * p[i];
}

__global__ void k_cg_finish(Status* st, int slot) {
  st->cg_iters[slot] = st->iters;
  if (st->breakdown || !st->all_done) st->converged = 0;
}

// ---------------------------------------------------- column-local CG step
// Every vector operation of a CG iteration except the Hessian product acts on one probe
// column j alone: alpha_j needs <p_j, q_j>, the residual test, the projection (a mean over
// the classes of each feature) and z_j = M^-1 r_j (one d x d product per class) stay inside
// the column.  A CG iteration is the product plus three small kernels (k_cg_col_alpha,
// k_cg_col_apply, k_cg_col_beta below) that keep the column vectors in LDS (FP64) and spread
// the block apply over classes; k_cg_col_init starts a solve with one block per column, and
// k_col_status folds the per-column flags into the status at each check point.  Used when
// (3 + kColSplit) d c doubles fit in LDS.

constexpr int kColThreads = 1024;
constexpr int kColSplit = 4;     // each output of the apply is summed in 4 pieces over b
constexpr int kApplyCols = 4;    // columns per block of k_cg_col_apply
constexpr int kColE = 3;         // column elements per thread in k_cg_col_alpha / _beta

int64_t col_cg_scratch(int d, int c, int s_max) {
  // the column-local path needs the init kernel's (3 + kColSplit) d c doubles in LDS
  // (so d c <= 2340), and at most kColE elements of a column per thread
  if ((int64_t)(3 + kColSplit) * d * c * 8 > 128 * 1024) return 0;
  if ((int64_t)d * c > (int64_t)kColE * kColThreads) return 0;
  return 2 * (int64_t)d * c * s_max;
}

__device__ __forceinline__ double block_sum_col(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kColThreads / 64; ++i) r += red[i];
  return r;
}

// z = M^-1 rs (both [c][d] in LDS, FP64), optionally projected before and after.
// zp: [kColSplit][c*d] LDS scratch for the partial dot products.
__device__ void col_apply(const double* __restrict__ Pinv, double* rs, double* zs, double* zp,
                          int d, int c, bool project) {
  const int n = d * c;
  if (project) {
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += rs[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) rs[k * d + a] -= m;
    }
    __syncthreads();
  }
  const int piece = (d + kColSplit - 1) / kColSplit;
  for (int w = threadIdx.x; w < kColSplit * n; w += blockDim.x) {
    const int q = w / n, e = w - q * n;
    const int k = e / d, a = e - k * d;
    const double* Pk = Pinv + (int64_t)k * d * d + a;
    const double* rk = rs + k * d;
    const int b0 = q * piece, b1 = min(d, b0 + piece);
    double acc = 0.0;
    for (int bb = b0; bb < b1; bb += 16) {
      // sixteen independent loads in flight before the products
      double pv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) pv[u] = bb + u < b1 ? Pk[(int64_t)(bb + u) * d] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (bb + u < b1) acc += pv[u] * rk[bb + u];
    }
    zp[w] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double z = 0.0;
#pragma unroll
    for (int q = 0; q < kColSplit; ++q) z += zp[q * n + e];
    zs[e] = z;
  }
  __syncthreads();
  if (project) {
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += zs[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) zs[k * d + a] -= m;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kColThreads) void k_cg_col_init(const T* __restrict__ B, T* __restrict__ xv,
                                                     T* __restrict__ r, T* __restrict__ p,
                                                     const double* __restrict__ Pinv, int d, int s,
                                                     int c, int project, double* rho,
                                                     double* bnorm, double* relres, int32_t* done,
                                                     Status* st) {
  extern __shared__ double sh[];
  __shared__ double red[kColThreads / 64];
  double* rs = sh;               // [c][d]
  double* zs = sh + d * c;       // [c][d]
  double* zp = zs + d * c;       // [kColSplit][c][d]
  const int j = blockIdx.x, n = d * c;
  const int64_t sc = (int64_t)s * c;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {   // (a, k), k fastest: coalesced rows
    const int a = e / c, k = e - a * c;
    rs[k * d + a] = (double)B[a * sc + (int64_t)j * c + k];
  }
  __syncthreads();
  if (project) {
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += rs[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) rs[k * d + a] -= m;
    }
    __syncthreads();
  }
  // r = b (projected), rounded to the working type as stored; x = 0
  double bb = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int a = e / c, k = e - a * c;
    const int64_t gi = a * sc + (int64_t)j * c + k;
    const T rv = (T)rs[k * d + a];
    r[gi] = rv;
    xv[gi] = T(0);
    rs[k * d + a] = (double)rv;
    bb += (double)rv * (double)rv;
  }
  bb = block_sum_col(bb, red);
  col_apply(Pinv, rs, zs, zp, d, c, project);
  double rz = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int a = e / c, k = e - a * c;
    const int64_t gi = a * sc + (int64_t)j * c + k;
    const T zv = (T)zs[k * d + a];
    p[gi] = zv;
    rz += (double)r[gi] * (double)zv;
  }
  rz = block_sum_col(rz, red);
  if (threadIdx.x == 0) {
    // an earlier failure (non-SPD block, breakdown in the previous solve) stops this solve
    const bool failed = st->breakdown != 0 || st->bad_block != INT_MAX;
    bnorm[j] = sqrt(bb);
    rho[j] = rz;
    done[j] = bb == 0.0 || failed;
    relres[j] = bb > 0.0 ? 1.0 : 0.0;
    if (j == 0) st->iters = 0;
  }
}

// One CG iteration of column j in three kernels around the block apply.  done_prev holds
// every column's flag after the previous iteration (read-only here); done_next receives this
// iteration's flags, so no block ever reads a flag another block of the same launch writes.
//
// k_cg_col_alpha (one block per column): alpha = rho / <p, q>, x += alpha p, r -= alpha q,
// projection of r, the residual test; an active column leaves its stored r, projected once
// more in FP64, in rd ([column][class][feature]).
// k_cg_col_apply (one block per class and group of columns): zd = P_k^-1 rd for the group,
// so each block of P^-1 is read once per group instead of once per column.
// k_cg_col_beta (one block per column): projection of z, rz = <r, z>, beta = rz / rho,
// p = z + beta p.
// The reductions keep one element per thread in the same order in all three, and the apply
// sums each output in kColSplit pieces over b exactly as col_apply does.
// One 32-bit word per column and iteration, so the host never sees half of it:
// (tag << 2) | (relative residual below the bf16x3 switch) << 1 | column stopped.
__device__ __forceinline__ void put_check(uint32_t* hword, int j, uint32_t tag, bool done,
                                          bool below) {
  if (hword) hword[j] = (tag << 2) | (below ? 2u : 0u) | (done ? 1u : 0u);
}

template <typename T>
__global__ __launch_bounds__(kColThreads) void k_cg_col_alpha(T* __restrict__ xv, T* __restrict__ r,
                                                      const T* __restrict__ p,
                                                      const T* __restrict__ q, int d, int s,
                                                      int c, int project, double tol, double* rho,
                                                      const double* bnorm, double* relres,
                                                      const int32_t* done_prev, int32_t* done_next,
                                                      double* __restrict__ rd, uint32_t* hword,
                                                      uint32_t tag, double res_switch,
                                                      Status* st) {
  // hword (may be null): this iteration's host-visible check word of each column, written on
  // every path so that the host finds all s words tagged
  extern __shared__ double sh[];
  __shared__ double red[kColThreads / 64];
  double* r0s = sh;   // [c][d]
  const int j = blockIdx.x, n = d * c;
  const int64_t sc = (int64_t)s * c;
  // Every global value of the step is loaded up front, before the flags are known (all in
  // bounds), so the step waits on memory once.  Element e = threadIdx.x + u kColThreads walks
  // (a, k) with k fastest: the c classes of a probe are contiguous in the block layout; the
  // LDS vectors keep the vec order k d + a.
  T pv[kColE], qv[kColE], rv[kColE], xw[kColE];
  int64_t gi[kColE];
  int li[kColE];
#pragma unroll
  for (int u = 0; u < kColE; ++u) {
    const int e = threadIdx.x + u * kColThreads;
    const int a = e / c, k = e - a * c;
    gi[u] = e < n ? a * sc + (int64_t)j * c + k : 0;
    li[u] = k * d + a;
    pv[u] = e < n ? p[gi[u]] : T(0);
    qv[u] = e < n ? q[gi[u]] : T(0);
    rv[u] = e < n ? r[gi[u]] : T(0);
    xw[u] = e < n ? xv[gi[u]] : T(0);
  }
  const double rho_j = rho[j], bn = bnorm[j], rel_prev = relres[j];
  const bool was_done = done_prev[j] != 0;
  if (skip_now(skip_all(done_prev, s))) {
    // nothing left: carry the flags forward so the next launch reads a current set
    if (threadIdx.x == 0) {
      done_next[j] = 1;
      put_check(hword, j, tag, true, rel_prev < res_switch);
    }
    return;
  }
  if (j == 0 && threadIdx.x == 0) st->iters += 1;
  if (was_done) {
    if (threadIdx.x == 0) {
      done_next[j] = 1;
      put_check(hword, j, tag, true, rel_prev < res_switch);
    }
    return;
  }
  double pq = 0.0;
#pragma unroll
  for (int u = 0; u < kColE; ++u)
    if (threadIdx.x + u * kColThreads < n) pq += (double)pv[u] * (double)qv[u];
  pq = block_sum_col(pq, red);
  if (!(pq > 0.0)) {   // breakdown: report it and freeze the column
    if (threadIdx.x == 0) {
      st->breakdown = 1;
      done_next[j] = 1;
      put_check(hword, j, tag, true, rel_prev < res_switch);
    }
    return;
  }
  const T at = (T)(rho_j / pq);
#pragma unroll
  for (int u = 0; u < kColE; ++u)
    if (threadIdx.x + u * kColThreads < n) {
      xv[gi[u]] = xw[u] + at * pv[u];
      r0s[li[u]] = (double)(rv[u] - at * qv[u]);
    }
  __syncthreads();
  if (project) {
    // r stays in the complement of {1_c (x) u} in exact arithmetic; remove the rounding
    // (the split products of BF16X3 leave ~1e-5 there, which the projected preconditioner
    // never searches, so it would floor the residual)
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += r0s[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) r0s[k * d + a] -= m;
    }
    __syncthreads();
  }
  double rr = 0.0;
#pragma unroll
  for (int u = 0; u < kColE; ++u)
    if (threadIdx.x + u * kColThreads < n) {
      const T rs = (T)r0s[li[u]];
      r[gi[u]] = rs;
      r0s[li[u]] = (double)rs;
      rr += (double)rs * (double)rs;
    }
  rr = block_sum_col(rr, red);
  const double rn = sqrt(rr);
  const bool now_done = rn <= tol * bn;
  if (threadIdx.x == 0) {
    const double rel = bn > 0.0 ? rn / bn : 0.0;
    done_next[j] = now_done;
    relres[j] = rel;
    put_check(hword, j, tag, now_done, rel < res_switch);
  }
  if (now_done) return;
  // the apply's input: the stored r, projected again in FP64 when asked
  double* rj = rd + (int64_t)j * n;
  if (project) {
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += r0s[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) rj[k * d + a] = r0s[k * d + a] - m;
    }
  } else {
    for (int e = threadIdx.x; e < n; e += blockDim.x) rj[e] = r0s[e];
  }
}

// zd[j][k][:] = P_k^-1 rd[j][k][:] for class k = blockIdx.x and the JT columns of group
// blockIdx.y; columns whose flag is set are skipped.  LDS: rd of the group (JT d doubles)
// and the kColSplit partial sums (kColSplit JT d doubles).
template <int JT>
__global__ __launch_bounds__(512) void k_cg_col_apply(const double* __restrict__ Pinv,
                                                      const double* __restrict__ rd,
                                                      double* __restrict__ zd, int d, int s,
                                                      int c, const int32_t* done) {
  extern __shared__ double sh[];
  double* rsh = sh;              // [JT][d]
  double* zp = sh + JT * d;      // [kColSplit][JT][d]
  const int k = blockIdx.x, j0 = blockIdx.y * JT;
  const int jn = min(JT, s - j0);
  const int n = d * c;
  const double* Pk = Pinv + (int64_t)k * d * d;
  const int piece = (d + kColSplit - 1) / kColSplit;
  // the first sixteen P^-1 values of this thread's first output, loaded together with the
  // flags and rd (the first pass of the loop below uses them)
  double pre[16];
  {
    const int w = threadIdx.x, qq = w / d, a = w - qq * d;
    const int b0 = qq * piece, b1 = min(d, b0 + piece);
#pragma unroll
    for (int u = 0; u < 16; ++u)
      pre[u] = w < kColSplit * d && b0 + u < b1 ? Pk[(int64_t)(b0 + u) * d + a] : 0.0;
  }
  int active = 0;
  for (int jj = 0; jj < jn; ++jj) active |= done[j0 + jj] == 0;
  if (!active) return;   // the same for every thread of the block
  for (int e = threadIdx.x; e < JT * d; e += blockDim.x) {
    const int jj = e / d, b = e - jj * d;
    rsh[e] = jj < jn ? rd[(int64_t)(j0 + jj) * n + (int64_t)k * d + b] : 0.0;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < kColSplit * d; w += blockDim.x) {
    const int qq = w / d, a = w - qq * d;
    const int b0 = qq * piece, b1 = min(d, b0 + piece);
    double acc[JT];
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) acc[jj] = 0.0;
    for (int bb = b0; bb < b1; bb += 16) {
      // sixteen independent loads in flight before the products
      double pv[16];
      const bool first = w == (int)threadIdx.x && bb == b0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        pv[u] = first ? pre[u] : (bb + u < b1 ? Pk[(int64_t)(bb + u) * d + a] : 0.0);
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (bb + u < b1) {
#pragma unroll
          for (int jj = 0; jj < JT; ++jj) acc[jj] += pv[u] * rsh[jj * d + bb + u];
        }
    }
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) zp[(qq * JT + jj) * d + a] = acc[jj];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < jn * d; e += blockDim.x) {
    const int jj = e / d, a = e - jj * d;
    double z = 0.0;
#pragma unroll
    for (int qq = 0; qq < kColSplit; ++qq) z += zp[(qq * JT + jj) * d + a];
    zd[(int64_t)(j0 + jj) * n + (int64_t)k * d + a] = z;
  }
}

template <typename T>
__global__ __launch_bounds__(kColThreads) void k_cg_col_beta(const T* __restrict__ r,
                                                     T* __restrict__ p,
                                                     const double* __restrict__ zd, int d,
                                                     int s, int c, int project, double* rho,
                                                     const int32_t* done) {
  extern __shared__ double sh[];
  __shared__ double red[kColThreads / 64];
  const int j = blockIdx.x, n = d * c;
  double* zs = sh;       // [c][d]
  double* r0s = sh + n;  // [c][d]
  const int64_t sc = (int64_t)s * c;
  const double* zj = zd + (int64_t)j * n;
  // all global loads first (in bounds whatever the flag), as in k_cg_col_alpha
  double zv[kColE];
  T rv[kColE], pv[kColE];
  int64_t gi[kColE];
  int li[kColE];
#pragma unroll
  for (int u = 0; u < kColE; ++u) {
    const int e = threadIdx.x + u * kColThreads;
    const int a = e / c, k = e - a * c;
    gi[u] = e < n ? a * sc + (int64_t)j * c + k : 0;
    li[u] = k * d + a;
    zv[u] = e < n ? zj[e] : 0.0;
    rv[u] = e < n ? r[gi[u]] : T(0);
    pv[u] = e < n ? p[gi[u]] : T(0);
  }
  const double rho_j = rho[j];
  if (done[j] != 0) return;
#pragma unroll
  for (int u = 0; u < kColE; ++u)
    if (threadIdx.x + u * kColThreads < n) {
      zs[threadIdx.x + u * kColThreads] = zv[u];
      r0s[li[u]] = (double)rv[u];
    }
  __syncthreads();
  if (project) {
    for (int a = threadIdx.x; a < d; a += blockDim.x) {
      double m = 0.0;
      for (int k = 0; k < c; ++k) m += zs[k * d + a];
      m /= c;
      for (int k = 0; k < c; ++k) zs[k * d + a] -= m;
    }
    __syncthreads();
  }
  // rz = <r, M^-1 r> with the stored (unprojected) r
  double rz = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) rz += r0s[e] * (double)(T)zs[e];
  rz = block_sum_col(rz, red);
  const double beta = rz / (rho_j != 0.0 ? rho_j : 1.0);
  const T bt = (T)beta;
#pragma unroll
  for (int u = 0; u < kColE; ++u)
    if (threadIdx.x + u * kColThreads < n) p[gi[u]] = (T)zs[li[u]] + bt * pv[u];
  if (threadIdx.x == 0) rho[j] = rz;
}

// Fold the per-column flags into the status (host check points and the end of a solve).
__global__ __launch_bounds__(256) void k_col_status(const int32_t* done, const double* relres, int s,
                                                    Status* st) {
  int ok = 1;
  double m = 0.0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    ok &= done[j] != 0;
    m = fmax(m, relres[j]);
  }
  const int all = __syncthreads_and(ok);
  m = block_max<256>(m);
  if (threadIdx.x == 0) {
    st->relres_max = m;
    st->all_done = all;
  }
}

// z = M^-1 r with M = blockdiag(P_k); projected: z = Pp M^-1 Pp r.
template <typename T>
static int apply_t(Ctx* x, const double* Pinv, const T* r, T* z, int s, bool project,
                   Skip skip, hipStream_t st) {
  const int d = x->d, c = x->c;
  const int64_t nds = (int64_t)d * s;
  if (project) {
    k_classmean<T><<<(unsigned)cdiv(nds, kRowWaves), 256, 0, st>>>(r, x->mean, d, s, c, skip);
    FIRAL_LAUNCHED();
  }
  // probes per group: all 16 of a Relax step's block while their LDS stays within 64 KB
  const double* mean = project ? x->mean : nullptr;
  if (d <= 512)
    papply_launch<T, 16>(Pinv, r, mean, z, d, s, c, skip, st);
  else if (d <= 2048)
    papply_launch<T, 4>(Pinv, r, mean, z, d, s, c, skip, st);
  else if (d <= 4096)
    papply_launch<T, 2>(Pinv, r, mean, z, d, s, c, skip, st);
  else
    return FIRAL_ENOTSUP;
  FIRAL_LAUNCHED();
  if (project) {
    k_project<T><<<(unsigned)cdiv(nds, kRowWaves), 256, 0, st>>>(z, z, d, s, c, skip);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ v, int64_t n, T value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = value;
}

// Wait until all s check words of one iteration carry its tag, then fold them: all columns
// stopped, all relative residuals below the bf16x3 switch.  The words arrive while the GPU
// runs ahead; after 1 ms of polling the host waits for the stream instead (long iterations),
// after which every word must be there.
static int poll_check(Ctx* x, const uint32_t* words, uint32_t tag, int s, hipStream_t st,
                      bool* all, bool* below) {
  const volatile uint32_t* w = words;
  auto tagged = [&]() {
    for (int j = 0; j < s; ++j)
      if ((w[j] >> 2) != tag) return false;
    return true;
  };
  const auto t0 = std::chrono::steady_clock::now();
  while (!tagged()) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(1)) {
      FIRAL_HIP(hipStreamSynchronize(st));
      if (!tagged()) {
        set_error("PCG check point: the column words of an iteration are missing");
        return FIRAL_EHIP;
      }
      break;
    }
  }
  bool a = true, b = true;
  for (int j = 0; j < s; ++j) {
    const uint32_t v = w[j];
    a = a && (v & 1u) != 0;
    b = b && (v & 2u) != 0;
  }
  *all = a;
  *below = b;
  return FIRAL_OK;
}

static int read_status(Ctx* x, hipStream_t st) {
  FIRAL_HIP(hipMemcpyAsync(x->status_host, x->status, sizeof(Status), hipMemcpyDeviceToHost, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  return FIRAL_OK;
}

template <typename T>
static int pcg_t(Ctx* x, const double* omega, double shift, const double* Pinv, const T* B,
                 T* Xsol, int s, double tol, int max_iter, uint32_t flags, int slot,
                 hipStream_t st) {
  const int d = x->d, c = x->c, P = x->col_parts;
  const int64_t n = (int64_t)d * s * c;
  const bool project = (flags & FIRAL_PCG_PROJECT) != 0;
  T* xv = (T*)x->cx;
  T* r = (T*)x->cr;
  T* z = (T*)x->cz;
  T* p = (T*)x->cp;
  T* q = (T*)x->cq;
  double* part0 = x->colpart;
  double* part1 = x->colpart + (int64_t)x->s_max * P;
  const Skip skip = skip_flag(&x->status->all_done);
  const unsigned nb = (unsigned)cdiv(n, 256);

  const size_t col_lds = (size_t)(3 + kColSplit) * d * c * sizeof(double);
  if (x->cgd && !x->force_multik) {
    // column-local CG: init, then per iteration the product and the three column kernels.
    // The iterate lives in the solution buffer itself when the caller gives one.
    if (Xsol && Xsol != B && Xsol != r && Xsol != p && Xsol != q) xv = Xsol;
    static DeviceOnce attr[2];
    if (!attr[sizeof(T) == 8].done()) {
      FIRAL_HIP(hipFuncSetAttribute((const void*)k_cg_col_init<T>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
      FIRAL_HIP(hipFuncSetAttribute((const void*)k_cg_col_alpha<T>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
      FIRAL_HIP(hipFuncSetAttribute((const void*)k_cg_col_beta<T>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
      FIRAL_HIP(hipFuncSetAttribute((const void*)k_cg_col_apply<1>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
      FIRAL_HIP(hipFuncSetAttribute((const void*)k_cg_col_apply<kApplyCols>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024));
      attr[sizeof(T) == 8].set();
    }
    double* rd = x->cgd;
    double* zd = x->cgd + (int64_t)d * c * x->s_max;
    const size_t alpha_lds = (size_t)d * c * sizeof(double);
    const size_t beta_lds = 2 * alpha_lds;
    // columns per apply block: kApplyCols while its LDS (rd and the partial sums of the
    // group) stays within 64 KiB, else one
    const int jt = (size_t)(1 + kColSplit) * kApplyCols * d * sizeof(double) <= 64 * 1024
                       ? kApplyCols : 1;
    const size_t apply_lds = (size_t)(1 + kColSplit) * jt * d * sizeof(double);
    const dim3 apply_grid((unsigned)c, (unsigned)cdiv(s, jt));
    int32_t* flags[2] = {x->done, x->done + x->s_max};
    k_cg_col_init<T><<<s, kColThreads, col_lds, st>>>(B, xv, r, p, Pinv, d, s, c, project, x->rho,
                                                      x->bnorm, x->relres, flags[0], x->status);
    FIRAL_LAUNCHED();
    // Mixed precision (BF16X3): bf16x3 products while every column's relative residual is
    // above bf3_switch, FP32 products once none is.  The switch keeps the operator error of
    // the split products from stalling the last iterations.
    const bool mixed = x->prec == FIRAL_BF16X3 && tol > 0.0 && !x->async;
    bool precise = false;
    // Host check points (tol > 0, not captured): iteration k's alpha kernel leaves one tagged
    // word per column in pinned host memory (slot k & 1).  Once iteration k is enqueued the
    // host polls iteration k-1's words, so the GPU always has an iteration queued and the
    // stream holds no extra packets.  When all columns have stopped, the one iteration
    // already enqueued runs kernels that skip on the device flags; a bf16x3 switch decided
    // at iteration k-1 takes effect from iteration k+1.
    const bool checks = tol > 0.0 && !x->async;
    const double res_switch = mixed ? x->bf3_switch : 0.0;
    uint32_t tags[2] = {0, 0};
    int launched = 0;
    while (launched < max_iter) {
      const int it = launched++;
      const int32_t* dp = flags[it & 1];
      int32_t* dn = flags[(it + 1) & 1];
      uint32_t* hw = checks ? x->chk_word_dev + (it & 1) * x->s_max : nullptr;
      tags[it & 1] = (++x->chk_tag) & 0x3fffffffu;
      if (tags[it & 1] == 0) tags[it & 1] = x->chk_tag = 1;   // zero marks an unwritten word
      FIRAL_CHECK(hvp_launch(x, omega, x->N, shift, p, q, s, skip_all(dp, s), st, precise));
      k_cg_col_alpha<T><<<s, kColThreads, alpha_lds, st>>>(xv, r, p, q, d, s, c, project, tol,
                                                           x->rho, x->bnorm, x->relres, dp, dn,
                                                           rd, hw, tags[it & 1], res_switch,
                                                           x->status);
      FIRAL_LAUNCHED();
      if (jt == kApplyCols)
        k_cg_col_apply<kApplyCols><<<apply_grid, 512, apply_lds, st>>>(Pinv, rd, zd, d, s, c, dn);
      else
        k_cg_col_apply<1><<<apply_grid, 512, apply_lds, st>>>(Pinv, rd, zd, d, s, c, dn);
      FIRAL_LAUNCHED();
      k_cg_col_beta<T><<<s, kColThreads, beta_lds, st>>>(r, p, zd, d, s, c, project, x->rho, dn);
      FIRAL_LAUNCHED();
      if (!checks || it == 0) continue;
      bool all = true, below = true;
      FIRAL_CHECK(poll_check(x, x->chk_word + ((it - 1) & 1) * x->s_max, tags[(it - 1) & 1], s,
                             st, &all, &below));
      if (all) break;
      if (mixed && below) precise = true;
    }
    // the status of the last enqueued iteration (all_done, relres_max) for k_cg_finish
    k_col_status<<<1, 256, 0, st>>>(flags[launched & 1], x->relres, s, x->status);
    FIRAL_LAUNCHED();
    k_cg_finish<<<1, 1, 0, st>>>(x->status, slot);
    FIRAL_LAUNCHED();
    if (Xsol && Xsol != xv)
      FIRAL_HIP(hipMemcpyAsync(Xsol, xv, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    return FIRAL_OK;
  }

  k_fill<T><<<nb, 256, 0, st>>>(xv, n, T(0));
  FIRAL_LAUNCHED();
  if (project) {
    k_project<T><<<(unsigned)cdiv((int64_t)d * s, kRowWaves), 256, 0, st>>>(B, r, d, s, c,
                                                                          skip_none());
    FIRAL_LAUNCHED();
  } else {
    FIRAL_HIP(hipMemcpyAsync(r, B, n * sizeof(T), hipMemcpyDeviceToDevice, st));
  }
  FIRAL_CHECK(apply_t<T>(x, Pinv, r, z, s, project, skip_none(), st));
  FIRAL_HIP(hipMemcpyAsync(p, z, n * sizeof(T), hipMemcpyDeviceToDevice, st));
  FIRAL_CHECK(coldot_launch(x, r, r, s, part0, skip_none(), st));
  FIRAL_CHECK(coldot_launch(x, r, z, s, part1, skip_none(), st));
  k_cg_init<<<1, 64, 0, st>>>(part0, part1, s, P, x->status, x->rho, x->bnorm, x->relres, x->done);
  FIRAL_LAUNCHED();

  const bool mixed = x->prec == FIRAL_BF16X3 && tol > 0.0 && !x->async;
  bool precise = false;
  const int check_every = tol > 0.0 && !x->async ? 4 : (max_iter > 0 ? max_iter : 1);
  int launched = 0;
  while (launched < max_iter) {
    const int batch = std::min(check_every, max_iter - launched);
    for (int it = 0; it < batch; ++it) {
      FIRAL_CHECK(hvp_launch(x, omega, x->N, shift, p, q, s, skip, st, precise));
      FIRAL_CHECK(coldot_launch(x, p, q, s, part0, skip, st));
      k_cg_alpha<<<1, 64, 0, st>>>(part0, s, P, x->status, x->rho, x->done, x->alpha);
      FIRAL_LAUNCHED();
      k_cg_update<T><<<nb, 256, 0, st>>>(xv, r, p, q, x->alpha, n, s, c, skip);
      FIRAL_LAUNCHED();
      if (project) {   // keep r in the projected space (removes rounding only)
        k_project<T><<<(unsigned)cdiv((int64_t)d * s, kRowWaves), 256, 0, st>>>(r, r, d, s, c,
                                                                              skip);
        FIRAL_LAUNCHED();
      }
      FIRAL_CHECK(coldot_launch(x, r, r, s, part1, skip, st));
      k_cg_done<<<1, 64, 0, st>>>(part1, s, P, x->status, x->bnorm, x->relres, x->done, tol);
      FIRAL_LAUNCHED();
      FIRAL_CHECK(apply_t<T>(x, Pinv, r, z, s, project, skip, st));
      FIRAL_CHECK(coldot_launch(x, r, z, s, part0, skip, st));
      k_cg_beta<<<1, 64, 0, st>>>(part0, s, P, x->status, x->rho, x->done, x->beta);
      FIRAL_LAUNCHED();
      k_cg_pupdate<T><<<nb, 256, 0, st>>>(p, z, x->beta, x->done, n, s, c, skip);
      FIRAL_LAUNCHED();
    }
    launched += batch;
    if (launched < max_iter) {
      FIRAL_CHECK(read_status(x, st));
      if (x->status_host->all_done) break;
      if (mixed && x->status_host->relres_max < x->bf3_switch) precise = true;
    }
  }
  k_cg_finish<<<1, 1, 0, st>>>(x->status, slot);
  FIRAL_LAUNCHED();
  if (Xsol != xv) FIRAL_HIP(hipMemcpyAsync(Xsol, xv, n * sizeof(T), hipMemcpyDeviceToDevice, st));
  return FIRAL_OK;
}

int pcg_launch(Ctx* x, const double* omega, double shift, const double* Pinv, const void* B,
               void* Xsol, int s, double tol, int max_iter, uint32_t flags, int slot,
               hipStream_t st) {
  if (x->prec == FIRAL_F64)
    return pcg_t<double>(x, omega, shift, Pinv, (const double*)B, (double*)Xsol, s, tol, max_iter,
                         flags, slot, st);
  return pcg_t<float>(x, omega, shift, Pinv, (const float*)B, (float*)Xsol, s, tol, max_iter,
                      flags, slot, st);
}

}  // namespace firal
