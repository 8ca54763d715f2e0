// Diagonal Round step of Approx-FIRAL (Algorithm 3, Section 3.2) on the rows of a context.
//
// Every d x d quantity is block diagonal with c blocks.  With Sigma_k = L_k L_k^T (the blocks
// of Sigma at the relaxed weights z_o, regulariser included), the round-t matrix
//   B_k = nu Sigma_k + eta (H)_k + (eta / b) (H_o)_k = L_k D_k L_k^T,
//   D_k = nu I + eta (C_k + O_k / b),   C_k = L_k^-1 (H)_k L_k^-T,   O_k = L_k^-1 (H_o)_k L_k^-T.
// The per-point objective of the Section 3.2 proposition needs, for every pool row x and class
// k, q1 = x^T B_k^-1 x and q2 = x^T B_k^-1 Sigma_k B_k^-1 x.  With u = L_k^-1 x and
// v = D_k^-1 u they are q1 = u . v and q2 = v . v, so one product per class,
// [u | v] = x^T [L_k^-T | (D_k^-1 L_k^-1)^T], scores every row (the L^-T half is triangular:
// its zero stages are skipped); the product's epilogue forms u . v, v . v and the class term
// g q2 / (1 + eta g q1) (g = h (1 - h)) without writing u or v.  The eigenvalues of
// (H~)_k = Sigma_k^-1/2 (H)_k Sigma_k^-1/2 that fix nu are those of C_k (similar matrices).
//
// A round: score (MFMA) -> sum over classes and argmax over the unselected rows (fixed order,
// lowest index on ties) -> update of C, (H) and the selection mask -> eigenvalues of C
// (Householder tridiagonalisation, then multisection on Sturm counts) -> nu_{t+1} (safeguarded
// Newton on Tr((nu I + eta C)^-2) = 1) -> D, its inverse (FP64 Cholesky) and the operand of
// round t + 1.  All state stays on the device and nothing is read back.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include <hip/hip_ext.h>

#include "common.h"

namespace firal {

namespace {

constexpr int kMaxD = 1024;         // d limit of the Round step (LDS rows of the update)
constexpr int kUpdSplit = 8;        // workgroups per class of the update, by row range
constexpr int kScoreTM = 64, kScoreTN = 64, kScoreTK = 16, kScorePad = 4;
constexpr int kTriThreads = 512;

__device__ __forceinline__ int64_t xcd_lid_r(int64_t b, int64_t n) {
  const int64_t q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// omega = [z ; 1] over the N rows (pool rows first)
__global__ void k_round_omega(const double* __restrict__ z, int64_t n_pool, int64_t N,
                              double* __restrict__ om) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) om[i] = i < n_pool ? z[i] : 1.0;
}

// Li_k = L_k^-1 (lower): column j by forward substitution, one column per thread.
__global__ __launch_bounds__(256) void k_tri_inv(const double* __restrict__ L,
                                                 double* __restrict__ Li, int d) {
  const int k = blockIdx.x;
  const double* Lk = L + (int64_t)k * d * d;
  double* Y = Li + (int64_t)k * d * d;
  for (int j0 = 0; j0 < d; j0 += blockDim.x) {
    const int j = j0 + threadIdx.x;
    const bool on = j < d;
    for (int i = 0; i < d; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int p = 0; p < i; ++p) acc -= Lk[(int64_t)i * d + p] * (on ? Y[(int64_t)p * d + j] : 0.0);
      if (on) Y[(int64_t)i * d + j] = acc / Lk[(int64_t)i * d + i];
    }
  }
}

// Batched C_k(i, j) = sum_p A_k(i, p) B_k(p, j) (i < M, j < N, p < K) with element strides;
// 32 x 32 output tiles through LDS, 2 x 2 outputs per thread.
struct BGemm {
  const double* A;
  int64_t sA;
  int64_t ai, ap;
  const double* B;
  int64_t sB;
  int64_t bp, bj;
  double* C;
  int64_t sC;
  int64_t ci, cj;
  int M, N, K;
};

__global__ __launch_bounds__(256) void k_bgemm(BGemm g) {
  __shared__ double As[32][33], Bs[32][33];
  const int tiles_n = (g.N + 31) / 32;
  const int ti = blockIdx.x / tiles_n, tj = blockIdx.x % tiles_n;
  const int64_t k = blockIdx.y;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const double* A = g.A + k * g.sA;
  const double* B = g.B + k * g.sB;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int p0 = 0; p0 < g.K; p0 += 32) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      const int r = e / 32, cc = e % 32;
      const int i = ti * 32 + r, p = p0 + cc;
      As[r][cc] = (i < g.M && p < g.K) ? A[i * g.ai + p * g.ap] : 0.0;
      const int pb = p0 + r, j = tj * 32 + cc;
      Bs[r][cc] = (pb < g.K && j < g.N) ? B[pb * g.bp + j * g.bj] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int pp = 0; pp < 32; ++pp) {
      const double a0 = As[2 * ty][pp], a1 = As[2 * ty + 1][pp];
      const double b0 = Bs[pp][2 * tx], b1 = Bs[pp][2 * tx + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  double* C = g.C + k * g.sC;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = ti * 32 + 2 * ty + u, j = tj * 32 + 2 * tx + v;
      if (i < g.M && j < g.N) C[i * g.ci + j * g.cj] = acc[u][v];
    }
}

// transposed copy of the c blocks L^-1 into the operand's u half: W_k[a][j] = Li_k[j][a]
__global__ void k_put_lit(const double* __restrict__ Li, int d, int c, int ldw,
                          double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (e >= (int64_t)c * dd) return;
  const int64_t k = e / dd;
  const int r = (int)(e - k * dd);
  const int a = r / d, j = r - (r / d) * d;
  W[(k * d + a) * ldw + j] = Li[k * dd + (int64_t)j * d + a];
}

// ------------------------------------------------------------------ eigenvalues
// Householder tridiagonalisation of each symmetric d x d block (Golub & Van Loan, Alg. 8.3.1):
// step j maps column j below the diagonal onto its first entry with P = I - beta v v^T and
// applies P A P to the trailing block as A - v w^T - w v^T with p = beta A v,
// w = p - (beta/2)(p . v) v.  The block is destroyed; diag[j] = a_jj, off[j] = a_{j+1,j} of
// the tridiagonal.  One workgroup per block, the block in global memory (d > 128; smaller
// blocks take k_tridiag_reg below).  diag and off are collected in LDS and written once at
// the end (a global store inside the loop would make every step's barrier wait for it).
__global__ __launch_bounds__(kTriThreads) void k_tridiag(double* __restrict__ A, int d,
                                                         double* __restrict__ diag,
                                                         double* __restrict__ off) {
  extern __shared__ double pp[];   // [4 d]: the four partial sums of each entry of A v
  __shared__ double v[kMaxD], p[kMaxD], dg[kMaxD], of[kMaxD];
  __shared__ double bc[2][2];
  const int blk = blockIdx.x, tid = threadIdx.x;
  A += (int64_t)blk * d * d;
  const int tc = tid & 31, tr = tid >> 5;   // 16 x 32 threads for the rank-2 update
  for (int j = 0; j + 2 < d; ++j) {
    const int r0 = j + 1, n2 = d - r0;   // trailing rows/columns r0 .. d-1
    double* bj = bc[j & 1];   // this step's scalars (alternate sets: no reader of the last
                              // step's set can see this step's values)
    // 1. wave 0: sigma = sum of squares below the subdiagonal entry, the reflector v and
    //    beta; bj[1] = 0 when column j is already reduced
    if (tid < 64) {
      double sg = 0.0;
      for (int i = 1 + tid; i < n2; i += 64) {
        const double x = A[(int64_t)(r0 + i) * d + j];
        sg += x * x;
      }
      sg = wave_sum(sg);
      const double x0 = A[(int64_t)r0 * d + j];
      if (tid == 0) dg[j] = A[(int64_t)j * d + j];
      if (sg == 0.0) {
        if (tid == 0) {
          of[j] = x0;
          bj[1] = 0.0;
        }
      } else {
        const double nx = sqrt(x0 * x0 + sg);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        const double v0 = x0 - alpha;
        for (int i = tid; i < n2; i += 64) v[i] = i == 0 ? v0 : A[(int64_t)(r0 + i) * d + j];
        if (tid == 0) {
          of[j] = alpha;
          bj[0] = 2.0 / (v0 * v0 + sg);
          bj[1] = 1.0;
        }
      }
    }
    __syncthreads();
    if (bj[1] == 0.0) continue;   // already tridiagonal in this column
    const double beta = bj[0];
    // 2. p = beta A_sub v by columns of the symmetric block, four threads per column: thread
    //    part k sums q = k mod 4 below the last multiple of four (part 0 also the rest), and
    //    the column's sum is (s0 + s1) + (s2 + s3)
    const int n4 = n2 & ~3;
    for (int t = tid; t < 4 * n2; t += kTriThreads) {
      const int i = t >> 2, part = t & 3;
      const double* col = A + (int64_t)r0 * d + r0 + i;
      double sk = 0.0;
      for (int q = part; q < n4; q += 4) sk = fma(col[(int64_t)q * d], v[q], sk);
      if (part == 0)
        for (int q = n4; q < n2; ++q) sk = fma(col[(int64_t)q * d], v[q], sk);
      pp[t] = sk;
    }
    __syncthreads();
    // 3. wave 0: p = beta A v, K = (beta / 2) p . v, p := w = p - K v
    if (tid < 64) {
      double pv = 0.0;
      for (int i = tid; i < n2; i += 64) {
        const double acc = (pp[4 * i] + pp[4 * i + 1]) + (pp[4 * i + 2] + pp[4 * i + 3]);
        p[i] = beta * acc;
        pv += beta * acc * v[i];
      }
      const double K = 0.5 * beta * wave_sum(pv);
      for (int i = tid; i < n2; i += 64) p[i] = p[i] - K * v[i];
    }
    __syncthreads();
    // 4. A_sub -= v w^T + w v^T
    for (int i = tr; i < n2; i += kTriThreads / 32) {
      double* arow = A + (int64_t)(r0 + i) * d + r0;
      const double vi = v[i], pi = p[i];
      for (int q = tc; q < n2; q += 32) arow[q] = arow[q] - vi * p[q] - pi * v[q];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (d >= 2) {
      dg[d - 2] = A[(int64_t)(d - 2) * d + d - 2];
      of[d - 2] = A[(int64_t)(d - 1) * d + d - 2];
    }
    dg[d - 1] = A[(int64_t)(d - 1) * d + d - 1];
    of[d - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < d; i += kTriThreads) {
    diag[(int64_t)blk * d + i] = dg[i];
    off[(int64_t)blk * d + i] = of[i];
  }
}

// The same reduction for d <= 128 with the block in registers: thread (ty, tx) of 16 x 16
// keeps A[ty + 16u][tx + 16w] (zero padding), and per step only column j, the partial sums
// of A v by thread column, and v and w go through LDS.  v and p are zero on the finished
// rows 0..j, so the rank-2 update leaves them alone.  The columns are walked in blocks of
// 16 (compile-time block index into the register tile).
struct TriLds {
  double* col;   // [128] column j of the current matrix
  double* v;     // [128]
  double* w;     // [128]
  double* part;  // [16][129] partial sums of A v, by thread column
  double* dg;    // [128]
  double* of;    // [128]
  double* bc;    // [2][2] beta and the "reflect" flag, alternate sets by step parity
};

template <int J, int D16>
__device__ __forceinline__ void tri_block(double (&a)[D16][D16], const TriLds& L, int d, int tid) {
  constexpr int PL = 129;
  const int ty = tid >> 4, tx = tid & 15;
  for (int jj = 0; jj < 16; ++jj) {
    const int j = 16 * J + jj;
    if (j + 2 >= d) return;   // uniform
    const int r0 = j + 1, n2 = d - r0;
    // 1. column j (rows below the diagonal) and the diagonal entry to LDS
    if (tx == jj) {
#pragma unroll
      for (int u = 0; u < D16; ++u) {
        const int i = ty + 16 * u;
        if (i > j) L.col[i] = a[u][J];
        if (i == j) L.dg[j] = a[u][J];
      }
    }
    __syncthreads();
    double* bj = L.bc + 2 * (j & 1);
    // 2. wave 0: sigma, the reflector v (zero on rows 0..j) and beta
    if (tid < 64) {
      double sg = 0.0;
      for (int i = r0 + 1 + tid; i < d; i += 64) sg += L.col[i] * L.col[i];
      sg = wave_sum(sg);
      const double x0 = L.col[r0];
      if (sg == 0.0) {
        if (tid == 0) {
          L.of[j] = x0;
          bj[1] = 0.0;
        }
      } else {
        const double nx = sqrt(x0 * x0 + sg);
        const double alpha = x0 >= 0.0 ? -nx : nx;
        const double v0 = x0 - alpha;
        for (int i = tid; i < 16 * D16; i += 64) L.v[i] = i < r0 || i >= d ? 0.0 : (i == r0 ? v0 : L.col[i]);
        if (tid == 0) {
          L.of[j] = alpha;
          bj[0] = 2.0 / (v0 * v0 + sg);
          bj[1] = 1.0;
        }
      }
    }
    __syncthreads();
    if (bj[1] == 0.0) continue;   // already tridiagonal in this column
    const double beta = bj[0];
    // 3. partial sums of A v over this thread's columns, for its rows
    double vq[D16];
#pragma unroll
    for (int w = 0; w < D16; ++w) vq[w] = L.v[tx + 16 * w];
#pragma unroll
    for (int u = 0; u < D16; ++u) {
      double sp = 0.0;
#pragma unroll
      for (int w = 0; w < D16; ++w) sp = fma(a[u][w], vq[w], sp);
      L.part[tx * PL + ty + 16 * u] = sp;
    }
    __syncthreads();
    // 4. wave 0: p = beta A v on the trailing rows (zero on 0..j), K = (beta/2) p . v,
    //    w = p - K v
    if (tid < 64) {
      double pv = 0.0;
      for (int i = tid; i < 16 * D16; i += 64) {
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) sum += L.part[t * PL + i];
        const double pi = i > j && i < d ? beta * sum : 0.0;
        L.w[i] = pi;
        pv += pi * L.v[i];
      }
      const double K = 0.5 * beta * wave_sum(pv);
      for (int i = tid; i < 16 * D16; i += 64) L.w[i] = L.w[i] - K * L.v[i];
    }
    __syncthreads();
    // 5. A -= v w^T + w v^T on this thread's entries
    double vi[D16], wi[D16], wq[D16];
#pragma unroll
    for (int u = 0; u < D16; ++u) {
      vi[u] = L.v[ty + 16 * u];
      wi[u] = L.w[ty + 16 * u];
      wq[u] = L.w[tx + 16 * u];
    }
#pragma unroll
    for (int u = 0; u < D16; ++u)
#pragma unroll
      for (int w = 0; w < D16; ++w) a[u][w] = a[u][w] - vi[u] * wq[w] - wi[u] * vq[w];
  }
}

template <int D16, int... Js>
__device__ __forceinline__ void tri_blocks(double (&a)[D16][D16], const TriLds& L, int d, int tid,
                                           std::integer_sequence<int, Js...>) {
  (tri_block<Js, D16>(a, L, d, tid), ...);
}

template <int D16>
__global__ __launch_bounds__(256) void k_tridiag_reg(double* __restrict__ A_all, int d,
                                                     double* __restrict__ diag,
                                                     double* __restrict__ off) {
  __shared__ double col[128], v[128], w[128], dg[128], of[128];
  __shared__ double part[16 * 129];
  __shared__ double bc[4];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const double* Ag = A_all + (int64_t)blk * d * d;
  double a[D16][D16];
#pragma unroll
  for (int u = 0; u < D16; ++u)
#pragma unroll
    for (int q = 0; q < D16; ++q) {
      const int i = ty + 16 * u, j = tx + 16 * q;
      a[u][q] = i < d && j < d ? Ag[(int64_t)i * d + j] : 0.0;
    }
  const TriLds L{col, v, w, part, dg, of, bc};
  tri_blocks<D16>(a, L, d, tid, std::make_integer_sequence<int, D16>{});
  // the last 2 x 2 (or 1 x 1) block
#pragma unroll
  for (int u = 0; u < D16; ++u)
#pragma unroll
    for (int q = 0; q < D16; ++q) {
      const int i = ty + 16 * u, j = tx + 16 * q;
      if (d >= 2 && i == d - 2 && j == d - 2) dg[d - 2] = a[u][q];
      if (d >= 2 && i == d - 1 && j == d - 2) of[d - 2] = a[u][q];
      if (i == d - 1 && j == d - 1) {
        dg[d - 1] = a[u][q];
        of[d - 1] = 0.0;
      }
    }
  __syncthreads();
  for (int i = tid; i < d; i += 256) {
    diag[(int64_t)blk * d + i] = dg[i];
    off[(int64_t)blk * d + i] = of[i];
  }
}

// Eigenvalues of each tridiagonal (diag a, off-diagonal e) on Sturm counts: the number of
// negative pivots of the LDL^T factorisation of T - x I is the number of eigenvalues below x
// (monotone in x).  Eigenvalue j starts from Gershgorin's bounds; S lanes of a wave share it
// and each evaluates one of S interior points of its bracket, a ballot finds the first point
// above the eigenvalue, and the bracket shrinks (S + 1)-fold per step (S = 1: bisection).
// Steps stop once the bracket is within 4 u ||T|| + 4 u |x| (u = 2^-53, the accuracy of the
// counts) or stops shrinking.  Pivots smaller than pivmin are replaced by -pivmin (LAPACK's
// safeguard).  Grid: (block, eigenvalue range of 256 / S).
template <int S>
__global__ __launch_bounds__(256) void k_sturm(const double* __restrict__ diag,
                                               const double* __restrict__ off, int d,
                                               double* __restrict__ lam) {
  constexpr int EPW = 256 / S;
  __shared__ double a[kMaxD], e2[kMaxD];
  __shared__ double bnd[3];
  const int blk = blockIdx.x, tid = threadIdx.x;
  const double* dg = diag + (int64_t)blk * d;
  const double* of = off + (int64_t)blk * d;
  double lo = INFINITY, hi = -INFINITY, emax = 0.0;
  for (int i = tid; i < d; i += blockDim.x) {
    a[i] = dg[i];
    const double el = i > 0 ? fabs(of[i - 1]) : 0.0, er = i + 1 < d ? fabs(of[i]) : 0.0;
    e2[i] = i + 1 < d ? of[i] * of[i] : 0.0;
    lo = fmin(lo, dg[i] - el - er);
    hi = fmax(hi, dg[i] + el + er);
    emax = fmax(emax, er * er);
  }
  lo = -block_max<256>(-lo);
  hi = block_max<256>(hi);
  emax = block_max<256>(emax);
  if (tid == 0) {
    bnd[0] = lo;
    bnd[1] = hi;
    bnd[2] = 2.2250738585072014e-308 * fmax(1.0, emax);
  }
  __syncthreads();
  const double L0 = bnd[0], H0 = bnd[1], pivmin = bnd[2];
  const double nrm = fmax(fabs(L0), fabs(H0));
  const double tol = 4.0 * 1.1102230246251565e-16 * nrm + pivmin;
  const int sl = tid % S, j = blockIdx.y * EPW + tid / S;
  const int gshift = (tid & 63) / S * S;        // first lane of this lane's group in the wave
  constexpr unsigned long long kGroupMask = S == 64 ? ~0ull : (1ull << (S % 64)) - 1;
  const bool on = j < d;
  double l = L0 - tol, u = H0 + tol;
  bool active = on;
  for (int it = 0; it < 200 && __any(active); ++it) {
    const double h = (u - l) / (S + 1);
    const double x = l + (sl + 1) * h;
    int cnt = 0;
    if (active) {
      double q = a[0] - x;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      for (int i = 1; i < d; ++i) {
        q = (a[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
      }
    }
    const uint64_t m = __ballot(active && cnt > j);
    if (active) {
      const unsigned long long bits = (m >> gshift) & kGroupMask;
      const double nl = bits == 0 ? l + S * h : (bits & 1ull ? l : l + (__ffsll(bits) - 1) * h);
      const double nu = bits == 0 ? u : l + __ffsll(bits) * h;
      if (!(nu - nl > tol + 4.0 * 1.1102230246251565e-16 * fmax(fabs(nl), fabs(nu))) ||
          (nl == l && nu == u))
        active = false;
      l = nl;
      u = nu;
    }
  }
  if (on && sl == 0) lam[(int64_t)blk * d + j] = 0.5 * (l + u);
}

// ------------------------------------------------------------------ nu
// nu_{t+1}: the root of phi(nu) = sum_kj (nu + eta lam_kj)^-2 = 1 on
// [1 - eta lam_min, sqrt(cd) - eta lam_min] (phi decreases there from >= 1 to <= 1).
// Newton steps on phi^-1/2 - 1 (close to linear in nu), replaced by bisection whenever they
// leave the bracket; stops when the bracket or the step vanishes.  One workgroup.
__global__ __launch_bounds__(1024) void k_round_nu(const double* __restrict__ lam, int64_t n,
                                                   double eta, double* __restrict__ nu_out) {
  __shared__ double bc[4];
  __shared__ int done;
  const int tid = threadIdx.x;
  double mn = INFINITY;
  for (int64_t e = tid; e < n; e += blockDim.x) mn = fmin(mn, lam[e]);
  const double negmax = block_max<1024>(-mn);
  if (tid == 0) bc[0] = -negmax;
  __syncthreads();
  mn = bc[0];
  double lo = 1.0 - eta * mn, hi = sqrt((double)n) - eta * mn;
  double nu = lo;
  if (tid == 0) done = 0;
  __syncthreads();
  for (int it = 0; it < 300; ++it) {
    double f = 0.0, fp = 0.0;
    for (int64_t e = tid; e < n; e += blockDim.x) {
      const double a = 1.0 / (nu + eta * lam[e]);
      const double a2 = a * a;
      f += a2;
      fp += a2 * a;
    }
    f = block_sum<1024>(f);
    fp = block_sum<1024>(fp);
    if (tid == 0) {
      const double phi = f, dphi = -2.0 * fp;
      if (phi > 1.0) lo = nu;
      else if (phi < 1.0) hi = nu;
      double nn;
      if (phi == 1.0) {
        nn = nu;
      } else {
        nn = nu + 2.0 * phi * (1.0 - sqrt(phi)) / dphi;
        if (!(nn > lo && nn < hi)) nn = 0.5 * (lo + hi);
      }
      if (nn == nu || !(hi - lo > 4e-16 * fabs(hi))) done = 1;
      bc[1] = nn;
      bc[2] = lo;
      bc[3] = hi;
    }
    __syncthreads();
    nu = bc[1];
    lo = bc[2];
    hi = bc[3];
    const int stop = done;
    __syncthreads();
    if (stop) break;
  }
  if (tid == 0) *nu_out = nu;
}

// The same iteration for up to 64 kNuPerLane eigenvalues in one wave: each lane keeps its
// eigenvalues in registers and every lane receives the wave-wide sums, so all lanes take
// the same steps and no barrier is needed.
constexpr int kNuPerLane = 32;
__global__ __launch_bounds__(64) void k_round_nu_wave(const double* __restrict__ lam, int n,
                                                      double eta, double* __restrict__ nu_out) {
  const int l = threadIdx.x;
  double lv[kNuPerLane];
  double mn = INFINITY;
#pragma unroll
  for (int u = 0; u < kNuPerLane; ++u) {
    const int e = l + 64 * u;
    lv[u] = e < n ? lam[e] : 0.0;
    if (e < n) mn = fmin(mn, lv[u]);
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));   // exact: any order
  double lo = 1.0 - eta * mn, hi = sqrt((double)n) - eta * mn;
  double nu = lo;
  for (int it = 0; it < 300; ++it) {
    double f = 0.0, fp = 0.0;
#pragma unroll
    for (int u = 0; u < kNuPerLane; ++u)
      if (l + 64 * u < n) {
        const double a = 1.0 / (nu + eta * lv[u]);
        const double a2 = a * a;
        f += a2;
        fp += a2 * a;
      }
    f = wave_sum(f);
    fp = wave_sum(fp);
    const double phi = f, dphi = -2.0 * fp;
    if (phi > 1.0) lo = nu;
    else if (phi < 1.0) hi = nu;
    double nn;
    if (phi == 1.0) {
      nn = nu;
    } else {
      nn = nu + 2.0 * phi * (1.0 - sqrt(phi)) / dphi;
      if (!(nn > lo && nn < hi)) nn = 0.5 * (lo + hi);
    }
    const bool stop = nn == nu || !(hi - lo > 4e-16 * fabs(hi));
    nu = nn;
    if (stop) break;
  }
  if (l == 0) *nu_out = nu;
}

// D_k = nu I + eta (C_k + O_k / b)
__global__ void k_form_d(const double* __restrict__ Cm, const double* __restrict__ Ot,
                         const double* __restrict__ nu_p, double eta, double inv_b, int d, int c,
                         double* __restrict__ Dm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (e >= (int64_t)c * dd) return;
  const int r = (int)(e % dd);
  const int i = r / d, j = r - (r / d) * d;
  Dm[e] = (i == j ? *nu_p : 0.0) + eta * (Cm[e] + Ot[e] * inv_b);
}

// FP32 copy of an FP64 array (the operand of the FP32 decision mode)
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// ------------------------------------------------------------------ scoring
// T[k][row] = g q2 / (1 + eta g q1) for the chunk's rows [r0, r0 + R) and class k, with
// q1 = u . v and q2 = v . v, [u | v] = x^T W_k, W_k = [L^-T | (D^-1 L^-1)^T] (d x 2 ldo, the
// halves at column offsets 0 and ldo; zero beyond d).  Workgroup: 64 rows x one class; it
// walks the class's d columns in tiles of 64, each tile accumulating the matching u and v
// columns (four waves of 32 x 32 each, 16x16x4 MFMA, stages of 16 k-rows double-buffered
// through LDS; a u block skips the stages below its triangle) and adds u . v and v . v per row
// to LDS slots.  Workgroup order (XCD-aware): row tile then class when all class operands
// fit in L2 together, else class then row tile.
// CT is the decision precision: every step from the products to the class term is computed
// in CT (FP64, or FP32 on the FP32 MFMA as the paper's single-precision implementation does).
// FP32 operands run four workgroups per CU, FP64 three (rows padded by two values instead of
// four so that three fit in LDS), both without scratch; the four k-steps of a stage are unrolled
// by two.  FP64 operands: the next stage's loads are issued before the current stage's products
// (raw values at clamped addresses) and staged after them, masked and converted to CT there, so
// that their latency is hidden behind the products (measured 548 -> 516 us a round at
// n = 50,000, d = 100, c = 10).  FP32 operands fetch the next stage after the products: their
// shorter products hide less, and the extra live registers made them 2-4% slower.
template <typename T, typename CT>
__global__ __launch_bounds__(256, sizeof(CT) == 4 ? 4 : 3) void k_round_score(const T* __restrict__ X,
                                                     const T* __restrict__ H, int64_t r0,
                                                     int64_t R, int d, int c,
                                                     const CT* __restrict__ W, int ldo,
                                                     double eta, int rows_major,
                                                     CT* __restrict__ Tout) {
  constexpr int TM = kScoreTM, TN = kScoreTN, TK = kScoreTK;
  constexpr int PAD = sizeof(CT) == 4 ? kScorePad : kScorePad / 2;   // FP64: three per CU fit
  constexpr int SA = TM + PAD, SB = TN + PAD;
  __shared__ CT As[2][TK][SA];
  __shared__ CT Bu[2][TK][SB];
  __shared__ CT Bv[2][TK][SB];
  __shared__ CT red[2][TM][2];
  typedef Mfma16<CT> MF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t ntr = (R + TM - 1) / TM;
  const int64_t lid = xcd_lid_r(blockIdx.x, (int64_t)gridDim.x);
  // rows_major: consecutive workgroups walk the classes of one row tile (the X tile is reused
  // from L2, every class operand stays resident); else the row tiles of one class (W_k stays
  // resident while X streams)
  const int k = rows_major ? (int)(lid % c) : (int)(lid / ntr);
  const int64_t row0 = (rows_major ? lid / c : lid - (int64_t)k * ntr) * TM;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const CT* Wk = W + (int64_t)k * d * 2 * ldo;
  const int nst = (d + TK - 1) / TK;
  const int nct = (d + TN - 1) / TN;

  for (int e = tid; e < 2 * TM * 2; e += 256) (&red[0][0][0])[e] = CT(0);

  // staging: A = 64 rows x 16 k, thread (row tid/16 + 16u, k tid%16), u = 0..3;
  // B = 16 k x 64 columns of each half, thread (k tid/64 + 4u, column tid%64)
  const int ak = tid & 15, ar = tid >> 4, bc = tid & 63, bk = tid >> 6;
  const int64_t arows = R - row0 - ar;              // rows of this thread's column in range
  constexpr bool kAhead = sizeof(CT) == 8;
  T ra[4];             // as stored (converted to CT when staged)
  CT rbu[4], rbv[4];
  unsigned ma = 0, mb = 0;   // bit u: value u in range
  int col0 = 0;
  auto load = [&](int st) {
    const int k0 = st * TK;
    const bool ka = k0 + ak < d;
    const bool cv = col0 + bc < d;
    ma = 0;
    mb = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool oka = ka && 16 * u < arows;
      ra[u] = X[oka ? (r0 + row0 + ar + 16 * u) * d + k0 + ak : 0];
      ma |= (unsigned)oka << u;
      const bool kb = k0 + bk + 4 * u < d && cv;
      const int64_t ob = kb ? ((int64_t)(k0 + bk + 4 * u) * 2 * ldo + col0 + bc) : 0;
      rbu[u] = Wk[ob];
      rbv[u] = Wk[ob + (kb ? ldo : 0)];
      mb |= (unsigned)kb << u;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[buf][ak][ar + 16 * u] = (ma >> u) & 1u ? (CT)ra[u] : CT(0);
      const bool kb = (mb >> u) & 1u;
      Bu[buf][bk + 4 * u][bc] = kb ? rbu[u] : CT(0);
      Bv[buf][bk + 4 * u][bc] = kb ? rbv[u] : CT(0);
    }
  };

  for (int ct = 0; ct < nct; ++ct) {
    col0 = ct * TN;
    typename MF::acc au[2][2], av[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) au[i][j] = av[i][j] = MF::zero();
    int jend[2];       // column block j is live and its u part has stages below k = jend
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int cb = col0 + wn + 16 * j;
      jend[j] = cb < d ? cb + 16 : 0;
    }
    load(0);
    store(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      const int k0 = st * TK;
      if constexpr (kAhead) {
        load(st + 1);   // past the last stage every value is out of range (stored as zero)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll 2
      for (int q = 0; q < TK / 4; ++q) {
        CT a[2], bu[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[buf][4 * q + g][wm + 16 * i + li];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          bu[j] = Bu[buf][4 * q + g][wn + 16 * j + li];
          bv[j] = Bv[buf][4 * q + g][wn + 16 * j + li];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if (jend[j] > 0) av[i][j] = MF::run(a[i], bv[j], av[i][j]);
            if (k0 < jend[j]) au[i][j] = MF::run(a[i], bu[j], au[i][j]);
          }
      }
      if constexpr (kAhead) {
        __builtin_amdgcn_sched_barrier(0);
        store(buf ^ 1);
      } else if (st + 1 < nst) {
        load(st + 1);
        store(buf ^ 1);
      }
      __syncthreads();
    }
    // this tile's u . v and v . v, summed over the lane's columns, then over the 16 lanes of
    // each row group; lane 0 of the group adds them to the row's slot
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        CT t1 = CT(0), t2 = CT(0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const CT uu = au[i][j][vv], vq = av[i][j][vv];
          t1 = fma(uu, vq, t1);
          t2 = fma(vq, vq, t2);
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          t1 += __shfl_xor(t1, o, 64);
          t2 += __shfl_xor(t2, o, 64);
        }
        if (li == 0) {
          const int row = wm + 16 * i + MF::row(g, vv);
          red[wave >> 1][row][0] += t1;
          red[wave >> 1][row][1] += t2;
        }
      }
  }
  __syncthreads();
  if (tid < TM) {
    const int64_t gr = row0 + tid;
    if (gr < R) {
      const CT q1 = red[0][tid][0] + red[1][tid][0];
      const CT q2 = red[0][tid][1] + red[1][tid][1];
      const double h = (double)H[(r0 + gr) * c + k];
      const CT gk = (CT)(h * (1.0 - h));        // g formed in FP64, then rounded to CT
      Tout[(int64_t)k * R + gr] = gk * q2 / (CT(1) + (CT)eta * gk * q1);
    }
  }
}

__device__ __forceinline__ bool better(double v1, int64_t i1, double v2, int64_t i2) {
  if (i1 < 0) return false;
  if (i2 < 0) return true;
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// r_i = sum_k T[k][i] in class order (in CT) for the chunk's rows; selected (and NaN) rows drop
// out.  Each block leaves its best (value, index) at part[r0 / 256 + block].
template <typename CT>
__global__ __launch_bounds__(256) void k_round_rsum(const CT* __restrict__ Tb, int64_t R,
                                                    int c, int64_t r0,
                                                    const int32_t* __restrict__ mask,
                                                    double* __restrict__ r_out,
                                                    double* __restrict__ pval,
                                                    int64_t* __restrict__ pidx) {
  __shared__ double sv[4];
  __shared__ int64_t si[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = -INFINITY;
  int64_t idx = -1;
  if (i < R) {
    CT s = CT(0);
    for (int k = 0; k < c; ++k) s += Tb[(int64_t)k * R + i];
    const int64_t gi = r0 + i;
    const bool sel = mask[gi] != 0;
    if (r_out) r_out[gi] = sel ? -INFINITY : (double)s;
    if (!sel && s == s) {
      v = (double)s;
      idx = gi;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_down(v, o, 64);
    const int64_t i2 = __shfl_down(idx, o, 64);
    if (better(v2, i2, v, idx)) {
      v = v2;
      idx = i2;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q)
      if (better(sv[q], si[q], v, idx)) {
        v = sv[q];
        idx = si[q];
      }
    pval[r0 / 256 + blockIdx.x] = v;
    pidx[r0 / 256 + blockIdx.x] = idx;
  }
}

// the best (value, index) over the block partials -> sel[t], smax[t] (-1 when nothing is left)
__global__ __launch_bounds__(1024) void k_round_pick(const double* __restrict__ pval,
                                                     const int64_t* __restrict__ pidx,
                                                     int64_t np, int64_t* __restrict__ sel,
                                                     double* __restrict__ smax, int t) {
  __shared__ double sv[16];
  __shared__ int64_t si[16];
  double v = -INFINITY;
  int64_t idx = -1;
  for (int64_t e = threadIdx.x; e < np; e += blockDim.x)
    if (better(pval[e], pidx[e], v, idx)) {
      v = pval[e];
      idx = pidx[e];
    }
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_down(v, o, 64);
    const int64_t i2 = __shfl_down(idx, o, 64);
    if (better(v2, i2, v, idx)) {
      v = v2;
      idx = i2;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 16; ++q)
      if (better(sv[q], si[q], v, idx)) {
        v = sv[q];
        idx = si[q];
      }
    sel[t] = idx;
    smax[t] = v;
  }
}

// The update for the row selected in round t, per class k: (H)_k += (H_o)_k / b + g x x^T and
// C_k += O_k / b + g u u^T with u = L_k^-1 x; a copy of C_k goes to the eigenvalue workspace;
// the row leaves the candidates.  Grid (c, kUpdSplit): each workgroup forms u for its class and
// updates one range of rows of the class's blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_round_update(
    const T* __restrict__ X, const T* __restrict__ H, int d, int c, double inv_b,
    const int64_t* __restrict__ sel, int t, const double* __restrict__ Li,
    const double* __restrict__ Ho, const double* __restrict__ Ot, double* __restrict__ Cm,
    double* __restrict__ Hacc, double* __restrict__ Ework, int32_t* __restrict__ mask,
    int32_t* __restrict__ err) {
  __shared__ double xs[kMaxD], us[kMaxD];
  const int k = blockIdx.x, part = blockIdx.y, tid = threadIdx.x;
  const bool lead = k == 0 && part == 0 && tid == 0;
  const int64_t i = sel[t];
  if (i < 0) {
    if (lead) err[0] = 1;
    return;
  }
  for (int a = tid; a < d; a += blockDim.x) xs[a] = (double)X[i * d + a];
  __syncthreads();
  const int64_t dd = (int64_t)d * d;
  const double* Lk = Li + k * dd;
  for (int a = tid; a < d; a += blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p <= a; ++p) acc += Lk[(int64_t)a * d + p] * xs[p];
    us[a] = acc;
  }
  __syncthreads();
  const double h = (double)H[i * c + k];
  const double gk = h * (1.0 - h);
  // this workgroup's rows of the class-k blocks (d <= kMaxD: an offset in a block fits int)
  const int rows = (d + kUpdSplit - 1) / kUpdSplit;
  const int a0 = part * rows, a1 = min(d, a0 + rows);
  for (int e = a0 * d + tid; e < a1 * d; e += blockDim.x) {
    const int a = e / d, bb = e - a * d;
    const int64_t s = k * dd + e;
    const double cn = Cm[s] + Ot[s] * inv_b + gk * us[a] * us[bb];
    Cm[s] = cn;
    Hacc[s] = Hacc[s] + Ho[s] * inv_b + gk * xs[a] * xs[bb];
    Ework[s] = cn;
  }
  if (lead) mask[i] = 1;
}

// min over all eigenvalues (one workgroup)
__global__ __launch_bounds__(1024) void k_min_eig(const double* __restrict__ lam, int64_t n,
                                                  double* __restrict__ out) {
  double mn = INFINITY;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) mn = fmin(mn, lam[e]);
  const double r = block_max<1024>(-mn);
  if (threadIdx.x == 0) *out = -r;
}

}  // namespace

// ------------------------------------------------------------------ state
struct Round {
  Ctx* x;                // borrowed; its profiling marks also bracket the scoring launches
  int d, c, ldo, b, t;
  int64_t n_pool, N, R, nparts;
  double eta;
  int fp32;              // decision precision FP32 (FIRAL_ROUND_FP32)
  double *omega, *Lf, *Li, *Ho, *Ot, *Cm, *Hacc, *Ew, *Dm, *Dinv, *tdiag, *toff, *lam, *W, *Tb,
      *pval, *nu, *smax, *gpart, *crit;
  float* Wf;             // FP32 copy of W in that mode
  int64_t *pidx, *sel;
  int32_t *mask, *flags, *tiles;   // flags: [0] Sigma_o not SPD, [1] no row left, [2] D not SPD
  int ntiles, splits;
};

static void free_round(Round* r) {
  void* bufs[] = {r->omega, r->Lf, r->Li, r->Ho, r->Ot, r->Cm, r->Hacc, r->Ew, r->Dm, r->Dinv,
                  r->tdiag, r->toff, r->lam, r->W, r->Tb, r->pval, r->nu, r->smax, r->gpart,
                  r->crit, r->Wf, r->pidx, r->sel, r->mask, r->flags, r->tiles};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete r;
}

static int rmalloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return FIRAL_ENOMEM;
  }
  return FIRAL_OK;
}

static int fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return FIRAL_OK;
  k_fill_f64<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(p, n, v);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}
static int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return FIRAL_OK;
  k_fill_i32<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(p, n, v);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

static int bgemm(const BGemm& g, int batch, hipStream_t st) {
  const unsigned tiles = (unsigned)(cdiv(g.M, 32) * cdiv(g.N, 32));
  k_bgemm<<<dim3(tiles, (unsigned)batch), 256, 0, st>>>(g);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// eigenvalues of the c blocks in A (destroyed) into lam (c x d)
static int eigvals_launch(Round* r, double* A, hipStream_t st) {
  const int d = r->d, c = r->c;
  // d <= 128: the block in registers; else the global-memory form (dynamic LDS: the 4 d
  // partial sums of A v)
  if (d <= 128) {
    switch ((d + 15) / 16) {
      case 1: k_tridiag_reg<1><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 2: k_tridiag_reg<2><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 3: k_tridiag_reg<3><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 4: k_tridiag_reg<4><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 5: k_tridiag_reg<5><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 6: k_tridiag_reg<6><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      case 7: k_tridiag_reg<7><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
      default: k_tridiag_reg<8><<<c, 256, 0, st>>>(A, d, r->tdiag, r->toff); break;
    }
  } else {
    k_tridiag<<<c, kTriThreads, 4 * (size_t)d * sizeof(double), st>>>(A, d, r->tdiag, r->toff);
  }
  FIRAL_LAUNCHED();
  // few eigenvalues: 64, 32 or 16 lanes share each one (65-, 33- or 17-section); many: one lane
  // each (bisection).  A whole wave per eigenvalue pays while it keeps the waves at about four
  // per SIMD or fewer (c d <= 4096); beyond that the doubled count work costs more than the
  // steps it saves.
  if ((int64_t)c * d <= 4096)
    k_sturm<64><<<dim3(c, (unsigned)cdiv(d, 256 / 64)), 256, 0, st>>>(r->tdiag, r->toff, d,
                                                                      r->lam);
  else if ((int64_t)c * d <= 32768)
    k_sturm<32><<<dim3(c, (unsigned)cdiv(d, 256 / 32)), 256, 0, st>>>(r->tdiag, r->toff, d,
                                                                      r->lam);
  else if ((int64_t)c * d <= 65536)
    k_sturm<16><<<dim3(c, (unsigned)cdiv(d, 256 / 16)), 256, 0, st>>>(r->tdiag, r->toff, d,
                                                                      r->lam);
  else
    k_sturm<1><<<dim3(c, (unsigned)cdiv(d, 256)), 256, 0, st>>>(r->tdiag, r->toff, d, r->lam);
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// the operand of the round that uses nu_p: D = nu I + eta (C + O / b), D^-1 (FP64 Cholesky),
// and the v half of W, (D^-1 L^-1)^T
static int round_operand(Round* r, const double* nu_p, hipStream_t st) {
  const int d = r->d, c = r->c;
  const int64_t dd = (int64_t)d * d;
  k_form_d<<<(unsigned)cdiv(c * dd, 256), 256, 0, st>>>(r->Cm, r->Ot, nu_p, r->eta, 1.0 / r->b,
                                                        d, c, r->Dm);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(chol_blocks_launch(r->Dm, r->Dinv, d, c, r->flags + 2, true, false, st));
  // F = D^-1 L^-1 stored transposed: W_k[a][ldo + j] = F_k[j][a]
  BGemm g{r->Dinv, dd, d, 1, r->Li, dd, d, 1, r->W + r->ldo, (int64_t)d * 2 * r->ldo, 1,
          2 * r->ldo, d, d, d};
  FIRAL_CHECK(bgemm(g, c, st));
  if (r->fp32) {
    const int64_t nw = (int64_t)c * d * 2 * r->ldo;
    k_to_f32<<<(unsigned)cdiv(nw, 256), 256, 0, st>>>(r->W, r->Wf, nw);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

// scores of every pool row at the current state into r_out (if non-null) and the block
// partials of the argmax
template <typename T, typename CT>
static int round_score_t(Round* r, const CT* W, double* r_out, hipStream_t st) {
  Ctx* x = r->x;
  const T* X = (const T*)x->X;
  const T* H = (const T*)x->H;
  CT* Tb = (CT*)r->Tb;
  for (int64_t r0 = 0; r0 < r->n_pool; r0 += r->R) {
    const int64_t R = std::min<int64_t>(r->R, r->n_pool - r0);
    const int64_t nwg = cdiv(R, kScoreTM) * r->c;
    hipEvent_t e0, e1;   // the kernel's own execution when profiling
    FIRAL_CHECK(prof_pair(r->x, FIRAL_PROF_ROUND_SCORE, &e0, &e1));
    // all c operands (d x 2 ldo each) within 2 MiB: walk the classes of a row tile together
    const int rows_major = (int64_t)r->c * r->d * 2 * r->ldo * sizeof(CT) <= ((int64_t)2 << 20);
    hipExtLaunchKernelGGL(k_round_score<T, CT>, dim3((unsigned)nwg), dim3(256), 0u, st, e0, e1,
                          0u, X, H, r0, R, r->d, r->c, W, r->ldo, r->eta, rows_major, Tb);
    FIRAL_LAUNCHED();
    k_round_rsum<CT><<<(unsigned)cdiv(R, 256), 256, 0, st>>>(Tb, R, r->c, r0, r->mask, r_out,
                                                             r->pval, r->pidx);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

static int round_score(Round* r, double* r_out, hipStream_t st) {
  const bool f64 = r->x->prec == FIRAL_F64;
  if (r->fp32)
    return f64 ? round_score_t<double, float>(r, r->Wf, r_out, st)
               : round_score_t<float, float>(r, r->Wf, r_out, st);
  return f64 ? round_score_t<double, double>(r, r->W, r_out, st)
             : round_score_t<float, double>(r, r->W, r_out, st);
}

static int round_step_launch(Round* r, hipStream_t st) {
  const int d = r->d, c = r->c, t = r->t;
  FIRAL_CHECK(round_score(r, nullptr, st));
  k_round_pick<<<1, 1024, 0, st>>>(r->pval, r->pidx, r->nparts, r->sel, r->smax, t);
  FIRAL_LAUNCHED();
  const Ctx* x = r->x;
  if (x->prec == FIRAL_F64)
    k_round_update<double><<<dim3(c, kUpdSplit), 256, 0, st>>>((const double*)x->X, (const double*)x->H, d, c,
                                              1.0 / r->b, r->sel, t, r->Li, r->Ho, r->Ot, r->Cm,
                                              r->Hacc, r->Ew, r->mask, r->flags + 1);
  else
    k_round_update<float><<<dim3(c, kUpdSplit), 256, 0, st>>>((const float*)x->X, (const float*)x->H, d, c,
                                             1.0 / r->b, r->sel, t, r->Li, r->Ho, r->Ot, r->Cm,
                                             r->Hacc, r->Ew, r->mask, r->flags + 1);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(eigvals_launch(r, r->Ew, st));
  if ((int64_t)c * d <= 64 * kNuPerLane)
    k_round_nu_wave<<<1, 64, 0, st>>>(r->lam, c * d, r->eta, r->nu + t + 1);
  else
    k_round_nu<<<1, 1024, 0, st>>>(r->lam, (int64_t)c * d, r->eta, r->nu + t + 1);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(round_operand(r, r->nu + t + 1, st));
  r->t = t + 1;
  return FIRAL_OK;
}

}  // namespace firal

using namespace firal;

#define RREQ(cond, ...)            \
  do {                             \
    if (!(cond)) {                 \
      set_error(__VA_ARGS__);      \
      return FIRAL_EINVAL;         \
    }                              \
  } while (0)

extern "C" int firal_round_create(firal_round* out, firal_ctx ctx, const double* z,
                                  double lambda, double eta, int32_t b, uint32_t flags,
                                  void* stream) {
  RREQ(out != nullptr && ctx != nullptr && z != nullptr, "firal_round_create: null argument");
  *out = nullptr;
  Ctx* x = C(ctx);
  RREQ(eta > 0.0 && std::isfinite(eta), "firal_round_create: eta must be positive");
  RREQ(lambda >= 0.0 && std::isfinite(lambda), "firal_round_create: lambda must be >= 0");
  RREQ(b >= 1 && (int64_t)b <= x->n_pool, "firal_round_create: b = %d outside [1, n_pool]", b);
  RREQ(x->d <= kMaxD, "firal_round_create: d = %d above the Round step's limit %d", x->d, kMaxD);
  RREQ(x->c <= 65535, "firal_round_create: c = %d above the Round step's limit 65535", x->c);
  RREQ((flags & ~FIRAL_ROUND_FP32) == 0, "firal_round_create: unknown flags 0x%x", flags);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(x->device));
  Round* r = new Round();
  r->x = x;
  r->d = x->d;
  r->c = x->c;
  r->ldo = (int)cdiv(x->d, 16) * 16;
  r->b = b;
  r->t = 0;
  r->n_pool = x->n_pool;
  r->N = x->N;
  r->eta = eta;
  r->fp32 = (flags & FIRAL_ROUND_FP32) != 0;
  const int d = r->d, c = r->c;
  // rows per scoring chunk: the class-term buffer c x R stays within 1 GiB
  const int64_t cap = std::max<int64_t>(256, (((int64_t)1 << 27) / c) / 256 * 256);
  r->R = std::min<int64_t>(cdiv(r->n_pool, 256) * 256, cap);
  r->nparts = cdiv(r->n_pool, 256);
  std::vector<int32_t> tiles;
  syrk_plan(FIRAL_F64, d, c, kGramClassic, 0, &tiles, &r->splits);
  r->ntiles = (int)(tiles.size() / 2);
  const int64_t dd = (int64_t)d * d;
  const int64_t nw = (int64_t)c * d * 2 * r->ldo;
  int rc = FIRAL_OK;
#define RALLOC(ptr, bytes)                                   \
  if (rc == FIRAL_OK) rc = rmalloc((void**)&(ptr), (bytes));
  RALLOC(r->omega, sizeof(double) * r->N);
  RALLOC(r->Lf, sizeof(double) * c * dd);
  RALLOC(r->Li, sizeof(double) * c * dd);
  RALLOC(r->Ho, sizeof(double) * c * dd);
  RALLOC(r->Ot, sizeof(double) * c * dd);
  RALLOC(r->Cm, sizeof(double) * c * dd);
  RALLOC(r->Hacc, sizeof(double) * c * dd);
  RALLOC(r->Ew, sizeof(double) * c * dd);
  RALLOC(r->Dm, sizeof(double) * c * dd);
  RALLOC(r->Dinv, sizeof(double) * c * dd);
  RALLOC(r->tdiag, sizeof(double) * c * d);
  RALLOC(r->toff, sizeof(double) * c * d);
  RALLOC(r->lam, sizeof(double) * c * d);
  RALLOC(r->W, sizeof(double) * nw);
  RALLOC(r->Tb, sizeof(double) * c * r->R);
  RALLOC(r->pval, sizeof(double) * r->nparts);
  RALLOC(r->pidx, sizeof(int64_t) * r->nparts);
  RALLOC(r->nu, sizeof(double) * (b + 1));
  RALLOC(r->smax, sizeof(double) * b);
  RALLOC(r->sel, sizeof(int64_t) * b);
  RALLOC(r->mask, sizeof(int32_t) * r->n_pool);
  RALLOC(r->flags, sizeof(int32_t) * 3);
  RALLOC(r->crit, sizeof(double));
  RALLOC(r->gpart, sizeof(double) * r->splits * c * dd);
  RALLOC(r->tiles, sizeof(int32_t) * tiles.size());
  if (r->fp32) RALLOC(r->Wf, sizeof(float) * nw);
#undef RALLOC
  if (rc != FIRAL_OK) {
    free_round(r);
    return rc;
  }
  auto fail = [&](int code) {
    free_round(r);
    return code;
  };
  if (hipMemcpyAsync(r->tiles, tiles.data(), sizeof(int32_t) * tiles.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipGetLastError();
    set_error("firal_round_create: copy failed");
    return fail(FIRAL_EHIP);
  }
#define RCHK(e)                    \
  do {                             \
    int rc_ = (e);                 \
    if (rc_ < 0) return fail(rc_); \
  } while (0)
  RCHK(fill_i32(r->flags, 1, INT_MAX, st));
  RCHK(fill_i32(r->flags + 1, 1, 0, st));
  RCHK(fill_i32(r->flags + 2, 1, INT_MAX, st));
  RCHK(fill_i32(r->mask, r->n_pool, 0, st));
  RCHK(fill(r->Cm, c * dd, 0.0, st));
  RCHK(fill(r->Hacc, c * dd, 0.0, st));
  RCHK(fill(r->W, nw, 0.0, st));
  k_fill_i64<<<(unsigned)cdiv(b, 256), 256, 0, st>>>(r->sel, b, -1);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(fill(r->nu, 1, std::sqrt((double)d * c), st));
  // Sigma_o blocks (rows weighted by [z ; 1], plus lambda I), factorised
  k_round_omega<<<(unsigned)cdiv(r->N, 256), 256, 0, st>>>(z, r->n_pool, r->N, r->omega);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(gram64_launch(x->prec, x->X, x->H, r->omega, r->N, d, c, r->tiles, r->ntiles, r->splits,
                     lambda, r->gpart, r->Lf, st));
  RCHK(chol_blocks_launch(r->Lf, r->Dinv, d, c, r->flags, false, true, st));
  // H_o blocks: the labeled rows with unit weight
  const size_t es = x->prec == FIRAL_F64 ? 8 : 4;
  RCHK(gram64_launch(x->prec, (const char*)x->X + es * r->n_pool * d,
                     (const char*)x->H + es * r->n_pool * c, nullptr, r->N - r->n_pool, d, c,
                     r->tiles, r->ntiles, r->splits, 0.0, r->gpart, r->Ho, st));
  k_tri_inv<<<c, 256, 0, st>>>(r->Lf, r->Li, d);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  // O_k = L^-1 H_o L^-T (Ew as the intermediate H_o L^-T)
  RCHK(bgemm(BGemm{r->Ho, dd, d, 1, r->Li, dd, 1, d, r->Ew, dd, d, 1, d, d, d}, c, st));
  RCHK(bgemm(BGemm{r->Li, dd, d, 1, r->Ew, dd, d, 1, r->Ot, dd, d, 1, d, d, d}, c, st));
  // the fixed u half of every class operand, then the first round's v half (nu_1 = sqrt(dc), C = 0)
  k_put_lit<<<(unsigned)cdiv(c * dd, 256), 256, 0, st>>>(r->Li, d, c, 2 * r->ldo, r->W);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(round_operand(r, r->nu, st));
  int32_t bad[3] = {INT_MAX, 0, INT_MAX};
  if (hipMemcpyAsync(bad, r->flags, sizeof(bad), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    set_error("firal_round_create: set-up failed");
    return fail(FIRAL_EHIP);
  }
  if (bad[0] != INT_MAX) {
    set_error("Sigma block %d of the Round step is not positive definite", bad[0]);
    return fail(FIRAL_ENOTSPD);
  }
  if (bad[2] != INT_MAX) {
    set_error("block %d of the first Round-step matrix is not positive definite", bad[2]);
    return fail(FIRAL_ENOTSPD);
  }
#undef RCHK
  *out = reinterpret_cast<firal_round>(r);
  return FIRAL_OK;
}

extern "C" int firal_round_step(firal_round round, int32_t rounds, void* stream) {
  RREQ(round != nullptr, "firal_round_step: null state");
  Round* r = reinterpret_cast<Round*>(round);
  RREQ(rounds >= 0 && r->t + (int64_t)rounds <= r->b,
       "firal_round_step: %d rounds requested, %d of b = %d left", rounds, r->b - r->t, r->b);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(r->x->device));
  for (int i = 0; i < rounds; ++i) FIRAL_CHECK(round_step_launch(r, st));
  return FIRAL_OK;
}

extern "C" int firal_round_scores(firal_round round, double* scores, void* stream) {
  RREQ(round != nullptr && scores != nullptr, "firal_round_scores: null argument");
  Round* r = reinterpret_cast<Round*>(round);
  FIRAL_HIP(hipSetDevice(r->x->device));
  return round_score(r, scores, (hipStream_t)stream);
}

extern "C" int firal_round_result(firal_round round, int64_t* selected, double* nu,
                                  double* score_max, int32_t* t, void* stream) {
  RREQ(round != nullptr, "firal_round_result: null state");
  Round* r = reinterpret_cast<Round*>(round);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(r->x->device));
  const int n = r->t;
  int32_t fl[3] = {INT_MAX, 0, INT_MAX};
  FIRAL_HIP(hipMemcpyAsync(fl, r->flags, sizeof(fl), hipMemcpyDeviceToHost, st));
  if (selected && n > 0)
    FIRAL_HIP(hipMemcpyAsync(selected, r->sel, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
  if (nu) FIRAL_HIP(hipMemcpyAsync(nu, r->nu, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, st));
  if (score_max && n > 0)
    FIRAL_HIP(hipMemcpyAsync(score_max, r->smax, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  if (t) *t = n;
  if (fl[1]) {
    set_error("Round step: no unselected pool row with a finite score was left");
    return FIRAL_EINVAL;
  }
  if (fl[2] != INT_MAX) {
    set_error("Round step: block %d of nu I + eta (C + O / b) is not positive definite", fl[2]);
    return FIRAL_ENOTSPD;
  }
  return FIRAL_OK;
}

extern "C" int firal_round_criterion(firal_round round, double* out, void* stream) {
  RREQ(round != nullptr && out != nullptr, "firal_round_criterion: null argument");
  Round* r = reinterpret_cast<Round*>(round);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(r->x->device));
  const int64_t n = (int64_t)r->c * r->d * r->d;
  FIRAL_HIP(hipMemcpyAsync(r->Ew, r->Hacc, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  FIRAL_CHECK(eigvals_launch(r, r->Ew, st));
  k_min_eig<<<1, 1024, 0, st>>>(r->lam, (int64_t)r->c * r->d, r->crit);
  FIRAL_LAUNCHED();
  FIRAL_HIP(hipMemcpyAsync(out, r->crit, sizeof(double), hipMemcpyDeviceToHost, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  return FIRAL_OK;
}

extern "C" int firal_round_destroy(firal_round round) {
  if (!round) return FIRAL_OK;
  Round* r = reinterpret_cast<Round*>(round);
  (void)hipSetDevice(r->x->device);
  free_round(r);
  return FIRAL_OK;
}

// The eta choice of the experiments section: the Round step for each eta of the list, keeping
// the selection whose (H)_k maximise min_k lambda_min((H)_k) (the first such eta on ties).
extern "C" int firal_round_eta_sweep(firal_ctx ctx, const double* z, double lambda,
                                     const double* etas, int32_t n_eta, int32_t b, uint32_t flags,
                                     int64_t* selected, double* criteria, int32_t* best,
                                     void* stream) {
  RREQ(ctx != nullptr && z != nullptr && etas != nullptr && selected != nullptr,
       "firal_round_eta_sweep: null argument");
  RREQ(n_eta >= 1, "firal_round_eta_sweep: n_eta = %d < 1", n_eta);
  RREQ(b >= 1, "firal_round_eta_sweep: b = %d < 1", b);
  std::vector<int64_t> sel((size_t)b);
  double best_crit = -INFINITY;
  int best_i = -1;
  for (int i = 0; i < n_eta; ++i) {
    firal_round r = nullptr;
    FIRAL_CHECK(firal_round_create(&r, ctx, z, lambda, etas[i], b, flags, stream));
    int rc = firal_round_step(r, b, stream);
    int32_t t = 0;
    if (rc >= 0) rc = firal_round_result(r, sel.data(), nullptr, nullptr, &t, stream);
    double crit = 0.0;
    if (rc >= 0) rc = firal_round_criterion(r, &crit, stream);
    (void)firal_round_destroy(r);
    if (rc < 0) return rc;
    if (criteria) criteria[i] = crit;
    if (best_i < 0 || crit > best_crit) {
      best_crit = crit;
      best_i = i;
      std::memcpy(selected, sel.data(), sizeof(int64_t) * (size_t)b);
    }
  }
  if (best) *best = best_i;
  return FIRAL_OK;
}
