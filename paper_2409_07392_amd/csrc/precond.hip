// Block-diagonal preconditioner of Definition 1 / eq. 12:
//   P_k = shift I_d + sum_i omega_i h_ik (1 - h_ik) x_i x_i^T,   k = 0..c-1,
// followed by an FP64 Cholesky factorisation P_k = L_k L_k^T and the explicit
// inverse P_k^-1 = L_k^-T L_k^-1 used by the PCG apply.
//
// The c weighted Gram matrices share the row data x_i: one wave owns a 16 x 16
// block pair (a-block >= b-block, the lower triangle) for a group of up to 16
// classes and a slice of rows; per group of 4 rows it loads x_i's two 16-wide
// pieces once and issues one MFMA per class with the A operand scaled by that
// class's weight u_ik = omega_i h_ik (1 - h_ik).  Slices of rows are reduced
// afterwards in FP64 in a fixed order.
#include <algorithm>
#include <climits>

#include "common.h"

namespace firal {

constexpr int kSyrkG = 16;   // classes per wave

__device__ __forceinline__ void pair_decode(int pair, int& ab, int& bb) {
  int a = (int)((sqrt(8.0 * pair + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= pair) ++a;
  while (a * (a + 1) / 2 > pair) --a;
  ab = a;
  bb = pair - a * (a + 1) / 2;
}

template <typename T>
__global__ __launch_bounds__(64) void k_syrk(const T* __restrict__ X, const T* __restrict__ H,
                                             const double* __restrict__ omega, int64_t N, int d,
                                             int c, int npairs, int64_t rows_per_split,
                                             T* __restrict__ part) {
  int ab, bb;
  pair_decode(blockIdx.x, ab, bb);
  const int kg0 = blockIdx.y * kSyrkG;
  const int ng = min(kSyrkG, c - kg0);
  const int64_t rb = (int64_t)blockIdx.z * rows_per_split;
  const int64_t re = rb + rows_per_split < N ? rb + rows_per_split : N;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int a = ab * 16 + li, b = bb * 16 + li;
  typedef Mfma16<T> M;
  typename M::acc acc[kSyrkG];
#pragma unroll
  for (int g = 0; g < kSyrkG; ++g) acc[g] = M::zero();

  for (int64_t r0 = rb; r0 < re; r0 += 4) {
    const int64_t r = r0 + lk;
    const bool ok = r < re;
    const T xa = (ok && a < d) ? X[r * d + a] : T(0);
    const T xb = (ok && b < d) ? X[r * d + b] : T(0);
    const T w = ok ? (omega ? (T)omega[r] : T(1)) : T(0);
    const T* hr = H + (ok ? r : 0) * c + kg0;
#pragma unroll
    for (int g = 0; g < kSyrkG; ++g) {
      if (g < ng) {
        const T h = ok ? hr[g] : T(0);
        const T u = w * h * (T(1) - h);
        acc[g] = M::run(u * xa, xb, acc[g]);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < kSyrkG; ++g) {
    if (g < ng) {
      T* o = part + (((int64_t)blockIdx.z * c + kg0 + g) * npairs + blockIdx.x) * 256;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[M::row(lk, v) * 16 + li] = acc[g][v];
    }
  }
}

// P[k][a][b] = sum_split part(lower-triangle element) + shift [a == b], FP64.
// Element (a, b) is always read from the (max, min) position so P is exactly symmetric.
template <typename T>
__global__ __launch_bounds__(256) void k_syrk_reduce(const T* __restrict__ part, int S, int c,
                                                     int d, int npairs, double shift,
                                                     double* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (idx >= (int64_t)c * dd) return;
  const int k = (int)(idx / dd);
  const int rem = (int)(idx % dd);
  int a = rem / d, b = rem % d;
  if (a < b) { const int t = a; a = b; b = t; }
  const int ab = a >> 4, bb = b >> 4;
  const int pair = ab * (ab + 1) / 2 + bb;
  const int within = (a & 15) * 16 + (b & 15);
  double acc = 0.0;
  for (int p = 0; p < S; ++p) acc += (double)part[(((int64_t)p * c + k) * npairs + pair) * 256 + within];
  P[idx] = acc + ((rem / d) == (rem % d) ? shift : 0.0);
}

// In-place right-looking Cholesky of block k (lower triangle); upper part zeroed.
// A non-positive (or NaN) pivot records k in *bad (smallest k wins) and stops the block.
__global__ __launch_bounds__(256) void k_chol(double* __restrict__ P, int d, int32_t* bad) {
  const int k = blockIdx.x;
  double* A = P + (int64_t)k * d * d;
  const int tid = threadIdx.x;
  for (int j = 0; j < d; ++j) {
    __syncthreads();
    const double piv = A[(int64_t)j * d + j];
    if (!(piv > 0.0)) {
      if (tid == 0) atomicMin(bad, k);
      return;
    }
    const double ljj = sqrt(piv);
    const double inv = 1.0 / ljj;
    __syncthreads();
    if (tid == 0) A[(int64_t)j * d + j] = ljj;
    for (int i = j + 1 + tid; i < d; i += blockDim.x) A[(int64_t)i * d + j] *= inv;
    __syncthreads();
    const int m = d - j - 1;
    for (int e = tid; e < m * m; e += blockDim.x) {
      const int ii = e / m, kk = e % m;
      if (kk <= ii) {
        const int i = j + 1 + ii, q = j + 1 + kk;
        A[(int64_t)i * d + q] -= A[(int64_t)i * d + j] * A[(int64_t)q * d + j];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < d * d; e += blockDim.x) {
    const int i = e / d, q = e % d;
    if (q > i) A[e] = 0.0;
  }
}

// Pinv_k = (L_k L_k^T)^-1, one column per thread: forward solve L y = e_j, then L^T x = y.
// All lanes walk the same (i, p) sequence (entries above the unit's row are zero), so the
// factor reads are uniform across the wave and the column reads/writes are coalesced.
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ L,
                                                  double* __restrict__ Pinv, int d,
                                                  const int32_t* bad) {
  if (*bad != INT_MAX) return;
  const int k = blockIdx.x;
  const double* Lk = L + (int64_t)k * d * d;
  double* Y = Pinv + (int64_t)k * d * d;
  for (int j0 = 0; j0 < d; j0 += blockDim.x) {
    const int j = j0 + threadIdx.x;
    const bool on = j < d;
    for (int i = 0; i < d; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int p = 0; p < i; ++p) acc -= Lk[(int64_t)i * d + p] * (on ? Y[(int64_t)p * d + j] : 0.0);
      if (on) Y[(int64_t)i * d + j] = acc / Lk[(int64_t)i * d + i];
    }
    for (int i = d - 1; i >= 0; --i) {
      double acc = on ? Y[(int64_t)i * d + j] : 0.0;
      for (int p = i + 1; p < d; ++p) acc -= Lk[(int64_t)p * d + i] * (on ? Y[(int64_t)p * d + j] : 0.0);
      if (on) Y[(int64_t)i * d + j] = acc / Lk[(int64_t)i * d + i];
    }
  }
}

// Cholesky factor and inverse of block k in one pass, the whole block held in registers.
// The symmetric sweep operator on pivot j maps a -> a - a_{:j} a_{j:} / a_jj off row/column j,
// a_{j:} / a_jj on them and -1/a_jj on the pivot; sweeping every pivot of an SPD matrix leaves
// -P^-1.  Before pivot j is swept its unswept column is the Schur complement, so
// L[i][j] = a_ij / sqrt(a_jj) (i >= j) is the Cholesky factor, and a_jj <= 0 means P is not SPD.
// Thread (ty, tx) of a TT x TT grid owns rows ty + TT u and columns tx + TT v (u, v < TB).
// L is written over P (P is read completely before the first pivot).
template <int TT, int TB>
__global__ __launch_bounds__(TT* TT) void k_sweep(double* __restrict__ P, double* __restrict__ Pinv,
                                                  int d, int32_t* bad) {
  const int kb = blockIdx.x;
  double* A0 = P + (int64_t)kb * d * d;
  double* Y = Pinv + (int64_t)kb * d * d;
  const int ty = threadIdx.x / TT, tx = threadIdx.x % TT;
  __shared__ double prow[TT * TB];
  double a[TB][TB];
#pragma unroll
  for (int u = 0; u < TB; ++u)
#pragma unroll
    for (int v = 0; v < TB; ++v) {
      const int i = ty + TT * u, q = tx + TT * v;
      a[u][v] = (i < d && q < d) ? A0[(int64_t)i * d + q] : 0.0;
    }
  __syncthreads();
  for (int j = 0; j < d; ++j) {
    const int uj = j / TT;
    if (ty == j % TT) {
#pragma unroll
      for (int u = 0; u < TB; ++u)
        if (u == uj) {
#pragma unroll
          for (int v = 0; v < TB; ++v) prow[tx + TT * v] = a[u][v];
        }
    }
    __syncthreads();
    const double piv = prow[j];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) atomicMin(bad, kb);
      return;
    }
    const double ip = 1.0 / piv;
    if (tx == 0) {
      const double sq = sqrt(piv);
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const int i = ty + TT * u;
        if (i >= j && i < d) A0[(int64_t)i * d + j] = i == j ? sq : prow[i] / sq;
      }
    }
    double pr[TB], pc[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) pr[u] = prow[ty + TT * u];
#pragma unroll
    for (int v = 0; v < TB; ++v) pc[v] = prow[tx + TT * v];
#pragma unroll
    for (int u = 0; u < TB; ++u)
#pragma unroll
      for (int v = 0; v < TB; ++v) {
        const int i = ty + TT * u, q = tx + TT * v;
        const double upd = a[u][v] - pr[u] * pc[v] * ip;
        const double onrow = (i == j) ? pc[v] * ip : pr[u] * ip;
        a[u][v] = (i == j && q == j) ? -ip : ((i == j || q == j) ? onrow : upd);
      }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < TB; ++u)
#pragma unroll
    for (int v = 0; v < TB; ++v) {
      const int i = ty + TT * u, q = tx + TT * v;
      if (i < d && q < d) {
        Y[(int64_t)i * d + q] = -a[u][v];
        if (q > i) A0[(int64_t)i * d + q] = 0.0;
      }
    }
}

typedef void (*SweepKernel)(double*, double*, int, int32_t*);

static SweepKernel pick_sweep(int d, int* threads) {
  if (d <= 128) {
    *threads = 256;
    switch ((d + 15) / 16) {
      case 1: return k_sweep<16, 1>;
      case 2: return k_sweep<16, 2>;
      case 3: return k_sweep<16, 3>;
      case 4: return k_sweep<16, 4>;
      case 5: return k_sweep<16, 5>;
      case 6: return k_sweep<16, 6>;
      case 7: return k_sweep<16, 7>;
      default: return k_sweep<16, 8>;
    }
  }
  if (d <= 256) {
    *threads = 1024;
    switch ((d + 31) / 32) {
      case 5: return k_sweep<32, 5>;
      case 6: return k_sweep<32, 6>;
      case 7: return k_sweep<32, 7>;
      default: return k_sweep<32, 8>;
    }
  }
  return nullptr;
}

__global__ void k_bad_reset(Status* st) { st->bad_block = INT_MAX; }

template <typename T>
static int precond_t(Ctx* x, const double* omega, double shift, hipStream_t st) {
  const int d = x->d, c = x->c;
  const int nb = (int)cdiv(d, 16);
  const int npairs = nb * (nb + 1) / 2;
  const int groups = (int)cdiv(c, kSyrkG);
  const int S = x->syrk_splits;
  const int64_t rps = cdiv(x->N, S);
  k_bad_reset<<<1, 1, 0, st>>>(x->status);
  FIRAL_LAUNCHED();
  k_syrk<T><<<dim3(npairs, groups, S), 64, 0, st>>>((const T*)x->X, (const T*)x->H, omega, x->N,
                                                   d, c, npairs, rps, (T*)x->syrk_part);
  FIRAL_LAUNCHED();
  const int64_t n = (int64_t)c * d * d;
  k_syrk_reduce<T><<<(unsigned)cdiv(n, 256), 256, 0, st>>>((const T*)x->syrk_part, S, c, d,
                                                           npairs, shift, x->P);
  FIRAL_LAUNCHED();
  int threads = 0;
  SweepKernel sw = pick_sweep(d, &threads);
  if (sw) {
    sw<<<c, threads, 0, st>>>(x->P, x->Pinv, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
  } else {
    k_chol<<<c, 256, 0, st>>>(x->P, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
    k_chol_inv<<<c, 256, 0, st>>>(x->P, x->Pinv, d, &x->status->bad_block);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

int precond_launch(Ctx* x, const double* omega, double shift, hipStream_t st) {
  if (x->prec == FIRAL_F64) return precond_t<double>(x, omega, shift, st);
  return precond_t<float>(x, omega, shift, st);
}

}  // namespace firal
