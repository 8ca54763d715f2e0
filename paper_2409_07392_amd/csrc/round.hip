// Diagonal Round step of Approx-FIRAL (Algorithm 3, Section 3.2) on the rows of a context.
//
// Every d x d quantity is block diagonal with c blocks.  With Sigma_k = L_k L_k^T (the blocks
// of Sigma at the relaxed weights z_o, regulariser included), the round-t matrix
//   B_k = nu Sigma_k + eta (H)_k + (eta / b) (H_o)_k = L_k D_k L_k^T,
//   D_k = nu I + eta E_k,   E_k = L_k^-1 ((H)_k + (H_o)_k / b) L_k^-T = Q_k Lambda_k Q_k^T.
// The per-point objective of the Section 3.2 proposition needs, for every pool row x and class
// k, q1 = x^T B_k^-1 x and q2 = x^T B_k^-1 Sigma_k B_k^-1 x.  With y = Q_k^T L_k^-1 x both are
// weighted sums of squares of one vector,
//   q1 = sum_j y_j^2 / (nu + eta lambda_kj),   q2 = sum_j y_j^2 / (nu + eta lambda_kj)^2,
// so one product per class, Y_k = X W_k with W_k = L_k^-T Q_k, scores every row; the
// product's epilogue forms the sums and the class term g q2 / (1 + eta g q1) (g = h(1 - h))
// without writing Y.  The eigenvalues of (H~)_k that fix nu are those of C_k = L_k^-1 (H)_k
// L_k^-T, which is similar to Sigma_k^-1/2 (H)_k Sigma_k^-1/2.
//
// A round: score (FP64 MFMA) -> sum over classes and argmax over the unselected rows (fixed
// order, lowest index on ties) -> update of C, (H) and the selection mask -> Jacobi
// eigensolves of C (values) and E (values and vectors) -> nu_{t+1} (safeguarded Newton on
// Tr((nu I + eta C)^-2) = 1) -> W and the weights of round t + 1.  All state stays on the
// device and nothing is read back.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "common.h"

namespace firal {

namespace {

constexpr int kMaxD = 512;          // d limit of the Round step (Jacobi pair tables, LDS rows)
constexpr int kScoreTM = 64, kScoreTN = 64, kScoreTK = 16, kScorePad = 4;

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
  int amod, bmod;   // batch k reads A block k % amod and B block k % bmod
};

__global__ __launch_bounds__(256) void k_bgemm(BGemm g) {
  __shared__ double As[32][33], Bs[32][33];
  const int tiles_n = (g.N + 31) / 32;
  const int ti = blockIdx.x / tiles_n, tj = blockIdx.x % tiles_n;
  const int64_t k = blockIdx.y;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const double* A = g.A + (k % g.amod) * g.sA;
  const double* B = g.B + (k % g.bmod) * g.sB;
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

// dst_k (m x m, zero padding beyond d) = sa * A_k + sb * B_k (d x d each; A or B may be null)
__global__ void k_pad_comb(const double* __restrict__ A, double sa, const double* __restrict__ B,
                           double sb, double* __restrict__ dst, int d, int m, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  if (e >= (int64_t)c * mm) return;
  const int64_t k = e / mm;
  const int r = (int)(e - k * mm);
  const int i = r / m, j = r - (r / m) * m;
  double v = 0.0;
  if (i < d && j < d) {
    const int64_t s = k * d * d + (int64_t)i * d + j;
    if (A) v += sa * A[s];
    if (B) v += sb * B[s];
  }
  dst[e] = v;
}

// ------------------------------------------------------------------ Jacobi eigensolver
// Cyclic two-sided Jacobi on symmetric m x m blocks (m even; a padding index d = m - 1 when d
// is odd never rotates).  Each sweep visits every pair once in m - 1 steps of m/2 disjoint
// pairs (round-robin: step r pairs (r, m-1) and ((r+p) mod (m-1), (r-p) mod (m-1)),
// p = 1..m/2-1).  A step computes each pair's rotation (c, s) zeroing a_pq (Golub & Van Loan,
// sym.schur2: tau = (a_qq - a_pp) / 2 a_pq, t = sign(tau) / (|tau| + sqrt(1 + tau^2))), then
// applies J^T A J block by block: each 2 x 2 block of rows of pair P and columns of pair R is
// computed once and written together with its transpose, so A stays exactly symmetric.
// Off-diagonal entries at or below 2.3e-16 ||A||_F (FP64 unit roundoff of the block's norm,
// evaluated at the start of each sweep) are zeroed without a rotation.  Sweeps
// stop once ||offdiag(A)||_F <= tol ||diag(A)||_2 (checked before each sweep), after a sweep
// without rotations, or after max_sweeps.  Blocks [0, n_vals) return eigenvalues only; later blocks also accumulate
// V <- V J (V starts at I; its columns are the eigenvectors).  SMEM: A (and V) are held in
// LDS for the whole solve.
template <bool SMEM, int NT>
__global__ __launch_bounds__(NT) void k_jacobi(double* __restrict__ A_all,
                                               double* __restrict__ V_all,
                                               double* __restrict__ lam_all, int m, int d,
                                               int n_vals, int v_given, int max_sweeps,
                                               double tol) {
  constexpr int kHalf = SMEM ? 64 : kMaxD / 2;
  extern __shared__ double dyn[];
  __shared__ double cs[kHalf], sn[kHalf], tn[kHalf];
  __shared__ int pp[kHalf], qq[kHalf], act[kHalf];
  __shared__ double stat[2];
  __shared__ int any_rot;
  int prev_rot = 1;
  const int blk = blockIdx.x, tid = threadIdx.x;
  const bool vecs = blk >= n_vals;
  const int mm = m * m;
  double* Ag = A_all + (int64_t)blk * mm;
  double* Vg = vecs ? V_all + (int64_t)(blk - n_vals) * mm : nullptr;
  double* A = Ag;
  double* V = Vg;
  if (SMEM) {
    A = dyn;
    V = vecs ? dyn + mm : nullptr;
    for (int e = tid; e < mm; e += NT) A[e] = Ag[e];
  }
  if (vecs) {
    if (v_given) {
      if (SMEM)
        for (int e = tid; e < mm; e += NT) V[e] = Vg[e];
    } else {
      for (int e = tid; e < mm; e += NT) V[e] = (e / m == e % m) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const int nb = m / 2, M = m - 1, half = nb / 2;
  // thread -> (pair myP, lane myq of stride nth): it updates the 2 x 2 blocks (myP, myP + dl)
  // for dl = myq, myq + nth, ... <= half, and rows myq, myq + nth, ... of V's two columns of
  // pair myP, loading the pair's rotation once
  const int nth = NT / nb;
  const int myP = tid % nb, myq = tid / nb;
  const bool worker = myq < nth;
  const int wave = tid >> 6, lane = tid & 63;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int i = wave; i < m; i += NT / 64)
      for (int j = lane; j < m; j += 64) {
        const double v = A[i * m + j];
        if (i == j) dg += v * v;
        else off += v * v;
      }
    off = block_sum<NT>(off);
    dg = block_sum<NT>(dg);
    if (tid == 0) {
      stat[0] = off;
      stat[1] = dg;
      any_rot = 0;
    }
    __syncthreads();
    const bool conv = stat[0] <= tol * tol * stat[1] || (sweep > 0 && prev_rot == 0);
    // entries at the rounding level of the whole block are zeroed, not rotated: in a degenerate
    // eigenspace (the zero eigenvalues of a rank-deficient block) rotations would only stir
    // that noise and the sweeps would not settle
    const double thr = 2.3e-16 * sqrt(stat[0] + stat[1]);
    __syncthreads();
    if (conv) break;
    for (int r = 0; r < M; ++r) {
      if (tid < nb) {
        const int P = tid;
        int p, q;
        if (P == 0) {
          p = r;
          q = M;
        } else {
          p = r + P;
          if (p >= M) p -= M;
          q = r - P;
          if (q < 0) q += M;
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0, t = 0.0;
        const double apq = A[p * m + q];
        const double app = A[p * m + p], aqq = A[q * m + q];
        int rot = 0;
        if (q < d && fabs(apq) > thr) {
          const double tau = (aqq - app) / (2.0 * apq);
          t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          any_rot = 1;
          rot = 1;
        }
        pp[P] = p;
        qq[P] = q;
        cs[P] = c;
        sn[P] = s;
        tn[P] = t;
        // 2: rotates; 1: only zeroes a_pq; 0: nothing to do
        act[P] = rot ? 2 : (apq != 0.0 ? 1 : 0);
      }
      __syncthreads();
      if (worker) {
        const int P = myP;
        const int aP = act[P], p = pp[P], q = qq[P];
        const double cP = cs[P], sP = sn[P];
        double* Ap = A + p * m;
        double* Aq = A + q * m;
        for (int dl = myq; dl <= half; dl += nth) {
          if ((nb & 1) == 0 && dl == half && P >= half) continue;
          if (dl == 0) {
            if (aP == 0) continue;
            const double apq = Ap[q], t = tn[P];
            Ap[p] = Ap[p] - t * apq;
            Aq[q] = Aq[q] + t * apq;
            Ap[q] = 0.0;
            Aq[p] = 0.0;
            continue;
          }
          int R = P + dl;
          if (R >= nb) R -= nb;
          if (aP < 2 && act[R] < 2) continue;   // both rotations are the identity
          const int r0 = pp[R], s0 = qq[R];
          const double cR = cs[R], sR = sn[R];
          const double a00 = Ap[r0], a01 = Ap[s0], a10 = Aq[r0], a11 = Aq[s0];
          const double b00 = cP * a00 - sP * a10, b01 = cP * a01 - sP * a11;
          const double b10 = sP * a00 + cP * a10, b11 = sP * a01 + cP * a11;
          const double e00 = cR * b00 - sR * b01, e01 = sR * b00 + cR * b01;
          const double e10 = cR * b10 - sR * b11, e11 = sR * b10 + cR * b11;
          Ap[r0] = e00;
          Ap[s0] = e01;
          Aq[r0] = e10;
          Aq[s0] = e11;
          A[r0 * m + p] = e00;
          A[s0 * m + p] = e01;
          A[r0 * m + q] = e10;
          A[s0 * m + q] = e11;
        }
        if (vecs && aP == 2) {
#pragma unroll 4
          for (int i = myq; i < m; i += nth) {
            double* Vi = V + i * m;
            const double v0 = Vi[p], v1 = Vi[q];
            Vi[p] = cP * v0 - sP * v1;
            Vi[q] = sP * v0 + cP * v1;
          }
        }
      }
      __syncthreads();
    }
    prev_rot = any_rot;
  }
  for (int i = tid; i < m; i += NT) lam_all[(int64_t)blk * m + i] = A[i * m + i];
  if (SMEM && vecs)
    for (int e = tid; e < mm; e += NT) Vg[e] = V[e];
}

size_t jacobi_smem_bytes(int m, bool vecs) { return (size_t)(vecs ? 2 : 1) * m * m * sizeof(double); }
// LDS per workgroup is 160 KiB; the kernel's static arrays (pair tables, reduction slots) take
// 2356 bytes when the blocks are held in LDS.
constexpr size_t kJacobiSmemMax = 160 * 1024 - 2560;

// Jacobi on n_vals value-only blocks followed by n_vec blocks with vectors (A_all holds them in
// that order; V_all the n_vec vector blocks).
int jacobi_launch(double* A_all, double* V_all, double* lam, int m, int d, int n_vals, int n_vec,
                  int v_given, hipStream_t st) {
  const int nblk = n_vals + n_vec;
  if (nblk == 0) return FIRAL_OK;
  const size_t smem = jacobi_smem_bytes(m, n_vec > 0);
  const int max_sweeps = 40;
  const double tol = 1e-14;
  if (smem <= kJacobiSmemMax && m / 2 <= 64) {
    static bool attr = false;
    if (!attr) {
      FIRAL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi<true, 1024>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kJacobiSmemMax));
      attr = true;
    }
    k_jacobi<true, 1024><<<nblk, 1024, smem, st>>>(A_all, V_all, lam, m, d, n_vals, v_given,
                                                   max_sweeps, tol);
  } else {
    k_jacobi<false, 512><<<nblk, 512, 0, st>>>(A_all, V_all, lam, m, d, n_vals, v_given,
                                               max_sweeps, tol);
  }
  FIRAL_LAUNCHED();
  return FIRAL_OK;
}

// ------------------------------------------------------------------ nu and weights
// nu_{t+1}: the root of phi(nu) = sum_kj (nu + eta lam_kj)^-2 = 1 on
// [1 - eta lam_min, sqrt(cd) - eta lam_min] (phi decreases there from >= 1 to <= 1).
// Newton steps on phi^-1/2 - 1 (close to linear in nu), replaced by bisection whenever they
// leave the bracket; stops when the bracket or the step vanishes.  One workgroup.
__global__ __launch_bounds__(1024) void k_round_nu(const double* __restrict__ lam, int m, int d,
                                                   int c, double eta, double* __restrict__ nu_out) {
  __shared__ double bc[4];
  __shared__ int done;
  const int n = c * d, tid = threadIdx.x;
  double mn = INFINITY;
  for (int e = tid; e < n; e += blockDim.x) mn = fmin(mn, lam[(int64_t)(e / d) * m + e % d]);
  // block min through the max of -x
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
    for (int e = tid; e < n; e += blockDim.x) {
      const double a = 1.0 / (nu + eta * lam[(int64_t)(e / d) * m + e % d]);
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

// weights of round t+1: w1_kj = 1 / (nu + eta lambda_kj), w2 = w1^2 (0 on padding columns)
__global__ void k_round_weights(const double* __restrict__ lamE, int m, int d, int c, int ldw,
                                const double* __restrict__ nu_p, double eta,
                                double* __restrict__ wts) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)c * ldw) return;
  const int64_t k = e / ldw;
  const int j = (int)(e - k * ldw);
  double w1 = 0.0;
  if (j < d) w1 = 1.0 / (*nu_p + eta * lamE[k * m + j]);
  wts[2 * e] = w1;
  wts[2 * e + 1] = w1 * w1;
}

// FP32 copy of an FP64 array (the operand and weights of the FP32 decision mode)
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// ------------------------------------------------------------------ scoring
// T[k][row] = g q2 / (1 + eta g q1) for the chunk's rows [r0, r0 + R) and class k, with
// (q1, q2) the weighted sums of squares of y = W_k^T x (see the file comment).  Workgroup: 64
// rows x one class; it walks the class's columns in tiles of 64 (four waves of 32 x 32, FP64
// 16x16x4 MFMA, stages of 16 k-rows double-buffered through LDS) and keeps the per-row sums in
// LDS.  Workgroups are ordered class-major (XCD-aware), so one XCD's tiles share W_k.
// CT is the decision precision: every step from y = W^T x to the class term is computed in CT
// (FP64, or FP32 on the FP32 MFMA as the paper's single-precision implementation does).
template <typename T, typename CT>
__global__ __launch_bounds__(256, 4) void k_round_score(const T* __restrict__ X,
                                                     const T* __restrict__ H, int64_t r0,
                                                     int64_t R, int d, int c,
                                                     const CT* __restrict__ W, int ldw,
                                                     const CT* __restrict__ wts, double eta,
                                                     CT* __restrict__ Tout) {
  constexpr int TM = kScoreTM, TN = kScoreTN, TK = kScoreTK;
  constexpr int SA = TM + kScorePad, SB = TN + kScorePad;
  __shared__ CT As[2][TK][SA];
  __shared__ CT Bs[2][TK][SB];
  __shared__ CT red[2][TM][2];
  typedef Mfma16<CT> MF;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t ntr = (R + TM - 1) / TM;
  const int64_t lid = xcd_lid_r(blockIdx.x, (int64_t)gridDim.x);
  const int k = (int)(lid / ntr);
  const int64_t row0 = (lid - (int64_t)k * ntr) * TM;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const CT* Wk = W + (int64_t)k * d * ldw;
  const CT* wk = wts + (int64_t)k * ldw * 2;
  const int nst = (d + TK - 1) / TK;
  const int nct = (ldw + TN - 1) / TN;

  // per-row sums of w1 y^2 and w2 y^2, one slot per column half of the workgroup
  for (int e = tid; e < 2 * TM * 2; e += 256) (&red[0][0][0])[e] = CT(0);

  // staging: A = 64 rows x 16 k, thread (row tid/16 + 16u, k tid%16), u = 0..3;
  // B = 16 k x 64 columns, thread (k tid/64 + 4u, column tid%64)
  const int ak = tid & 15, ar = tid >> 4, bc = tid & 63, bk = tid >> 6;
  const T* xa = X + (r0 + row0 + ar) * d + ak;
  const int64_t arows = R - row0 - ar;              // rows of this thread's column in range
  const CT* wb = Wk + (int64_t)bk * ldw + bc;
  CT ra[4], rb[4];
  int col0 = 0;
  auto load = [&](int st) {
    const int k0 = st * TK;
    const bool ka = k0 + ak < d;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ra[u] = (ka && 16 * u < arows) ? (CT)xa[(int64_t)16 * u * d + k0] : CT(0);
      rb[u] = (k0 + bk + 4 * u < d && col0 + bc < ldw) ? wb[(int64_t)(k0 + 4 * u) * ldw + col0]
                                                        : CT(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[buf][ak][ar + 16 * u] = ra[u];
      Bs[buf][bk + 4 * u][bc] = rb[u];
    }
  };

  for (int ct = 0; ct < nct; ++ct) {
    col0 = ct * TN;
    typename MF::acc acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = MF::zero();
    bool jon[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) jon[j] = col0 + wn + 16 * j < ldw;
    load(0);
    store(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      if (st + 1 < nst) load(st + 1);
#pragma unroll
      for (int q = 0; q < TK / 4; ++q) {
        CT av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = As[buf][4 * q + g][wm + 16 * i + li];
#pragma unroll
        for (int j = 0; j < 2; ++j) bv[j] = Bs[buf][4 * q + g][wn + 16 * j + li];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            if (jon[j]) acc[i][j] = MF::run(av[i], bv[j], acc[i][j]);
      }
      if (st + 1 < nst) store(buf ^ 1);
      __syncthreads();
    }
    // this tile's weighted squares, summed over the lane's columns, then over the 16 lanes
    // of each row group; lane 0 of the group adds them to the row's slot
    CT w1[2], w2[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wn + 16 * j + li;
      w1[j] = jon[j] ? wk[2 * col] : CT(0);
      w2[j] = jon[j] ? wk[2 * col + 1] : CT(0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        CT t1 = CT(0), t2 = CT(0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const CT y2 = acc[i][j][v] * acc[i][j][v];
          t1 = fma(w1[j], y2, t1);
          t2 = fma(w2[j], y2, t2);
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          t1 += __shfl_xor(t1, o, 64);
          t2 += __shfl_xor(t2, o, 64);
        }
        if (li == 0) {
          const int row = wm + 16 * i + MF::row(g, v);
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
// C_k += O_k / b + g u u^T with u = L_k^-1 x; the Jacobi inputs of the round (C_k, and
// E_k = C_k + O_k / b) are written padded to m x m; the row leaves the candidates.
template <typename T>
__global__ __launch_bounds__(256) void k_round_update(
    const T* __restrict__ X, const T* __restrict__ H, int d, int c, int m, double inv_b,
    const int64_t* __restrict__ sel, int t, const double* __restrict__ Li,
    const double* __restrict__ Ho, const double* __restrict__ Ot, double* __restrict__ Cm,
    double* __restrict__ Hacc, double* __restrict__ JA, int32_t* __restrict__ mask,
    int32_t* __restrict__ err) {
  __shared__ double xs[kMaxD], us[kMaxD];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int64_t i = sel[t];
  if (i < 0) {
    if (k == 0 && tid == 0) err[0] = 1;
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
  const int64_t mm = (int64_t)m * m;
  double* JC = JA + (int64_t)k * mm;
  double* JE = JA + ((int64_t)c + k) * mm;
  for (int64_t e = tid; e < mm; e += blockDim.x) {
    const int a = (int)(e / m), bb = (int)(e - (e / m) * m);
    if (a < d && bb < d) {
      const int64_t s = k * dd + (int64_t)a * d + bb;
      const double o = Ot[s];
      const double cn = Cm[s] + o * inv_b + gk * us[a] * us[bb];
      Cm[s] = cn;
      Hacc[s] = Hacc[s] + Ho[s] * inv_b + gk * xs[a] * xs[bb];
      JC[e] = cn;
      JE[e] = cn + o * inv_b;
    } else {
      JC[e] = 0.0;
      JE[e] = 0.0;
    }
  }
  if (k == 0 && tid == 0) mask[i] = 1;
}

// min over the c blocks' d eigenvalues (one workgroup)
__global__ __launch_bounds__(1024) void k_min_eig(const double* __restrict__ lam, int m, int d,
                                                  int c, double* __restrict__ out) {
  double mn = INFINITY;
  for (int e = threadIdx.x; e < c * d; e += blockDim.x)
    mn = fmin(mn, lam[(int64_t)(e / d) * m + e % d]);
  const double r = block_max<1024>(-mn);
  if (threadIdx.x == 0) *out = -r;
}

}  // namespace

// ------------------------------------------------------------------ state
struct Round {
  Ctx* x;                // borrowed; its profiling marks also bracket the scoring launches
  int d, c, m, ldw, b, t;
  int64_t n_pool, N, R, nparts;
  double eta;
  double *omega, *Lf, *Li, *Ho, *Ot, *Cm, *Hacc, *JA, *JV, *JT, *lam, *W, *wts, *Tb, *pval, *nu,
      *smax, *gpart, *crit;
  int64_t *pidx, *sel;
  int32_t *mask, *flags, *tiles;
  int ntiles, splits;
  int fp32;                // decision precision FP32 (FIRAL_ROUND_FP32)
  float *Wf, *wtsf;        // FP32 copies of W and the weights in that mode
};

static void free_round(Round* r) {
  void* bufs[] = {r->omega, r->Lf, r->Li, r->Ho, r->Ot, r->Cm, r->Hacc, r->JA, r->JV, r->JT, r->lam,
                  r->W, r->wts, r->Tb, r->pval, r->nu, r->smax, r->gpart, r->crit, r->pidx,
                  r->sel, r->mask, r->flags, r->tiles, r->Wf, r->wtsf};
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

// W_k = L_k^-T Q_k (Q_k: the first d columns of block k of JV) and the weights for nu_p
static int round_operand(Round* r, const double* nu_p, hipStream_t st) {
  const int d = r->d, c = r->c, m = r->m;
  const int64_t dd = (int64_t)d * d, mm = (int64_t)m * m;
  k_round_weights<<<(unsigned)cdiv((int64_t)c * r->ldw, 256), 256, 0, st>>>(
      r->lam + (int64_t)c * m, m, d, c, r->ldw, nu_p, r->eta, r->wts);
  FIRAL_LAUNCHED();
  BGemm g{r->Li, dd, 1, d, r->JV, mm, m, 1, r->W, (int64_t)d * r->ldw, r->ldw, 1, d, d, d,
          INT_MAX, INT_MAX};
  FIRAL_CHECK(bgemm(g, c, st));
  if (r->fp32) {
    const int64_t nw = (int64_t)c * d * r->ldw, nt = (int64_t)c * r->ldw * 2;
    k_to_f32<<<(unsigned)cdiv(nw, 256), 256, 0, st>>>(r->W, r->Wf, nw);
    FIRAL_LAUNCHED();
    k_to_f32<<<(unsigned)cdiv(nt, 256), 256, 0, st>>>(r->wts, r->wtsf, nt);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

// scores of every pool row at the current state into r_out (if non-null) and the block
// partials of the argmax
template <typename T, typename CT>
static int round_score_t(Round* r, const CT* W, const CT* wts, double* r_out, hipStream_t st) {
  const Ctx* x = r->x;
  const T* X = (const T*)x->X;
  const T* H = (const T*)x->H;
  CT* Tb = (CT*)r->Tb;
  for (int64_t r0 = 0; r0 < r->n_pool; r0 += r->R) {
    const int64_t R = std::min<int64_t>(r->R, r->n_pool - r0);
    const int64_t nwg = cdiv(R, kScoreTM) * r->c;
    FIRAL_CHECK(prof_mark(r->x, st, true));
    k_round_score<T, CT><<<(unsigned)nwg, 256, 0, st>>>(X, H, r0, R, r->d, r->c, W, r->ldw, wts,
                                                        r->eta, Tb);
    FIRAL_LAUNCHED();
    FIRAL_CHECK(prof_mark(r->x, st, false));
    k_round_rsum<CT><<<(unsigned)cdiv(R, 256), 256, 0, st>>>(Tb, R, r->c, r0, r->mask, r_out,
                                                             r->pval, r->pidx);
    FIRAL_LAUNCHED();
  }
  return FIRAL_OK;
}

static int round_score(Round* r, double* r_out, hipStream_t st) {
  const bool f64 = r->x->prec == FIRAL_F64;
  if (r->fp32)
    return f64 ? round_score_t<double, float>(r, r->Wf, r->wtsf, r_out, st)
               : round_score_t<float, float>(r, r->Wf, r->wtsf, r_out, st);
  return f64 ? round_score_t<double, double>(r, r->W, r->wts, r_out, st)
             : round_score_t<float, double>(r, r->W, r->wts, r_out, st);
}

static int round_step_launch(Round* r, hipStream_t st) {
  const int d = r->d, c = r->c, m = r->m, t = r->t;
  FIRAL_CHECK(round_score(r, nullptr, st));
  k_round_pick<<<1, 1024, 0, st>>>(r->pval, r->pidx, r->nparts, r->sel, r->smax, t);
  FIRAL_LAUNCHED();
  const Ctx* x = r->x;
  if (x->prec == FIRAL_F64)
    k_round_update<double><<<c, 256, 0, st>>>((const double*)x->X, (const double*)x->H, d, c, m,
                                              1.0 / r->b, r->sel, t, r->Li, r->Ho, r->Ot, r->Cm,
                                              r->Hacc, r->JA, r->mask, r->flags + 1);
  else
    k_round_update<float><<<c, 256, 0, st>>>((const float*)x->X, (const float*)x->H, d, c, m,
                                             1.0 / r->b, r->sel, t, r->Li, r->Ho, r->Ot, r->Cm,
                                             r->Hacc, r->JA, r->mask, r->flags + 1);
  FIRAL_LAUNCHED();
  // both eigenproblems of the round in the previous round's eigenbasis Q (JV):
  // JA_k <- Q^T JA_k Q, so they start close to diagonal; E's rotations accumulate onto Q
  const int64_t mm = (int64_t)m * m;
  FIRAL_CHECK(bgemm(BGemm{r->JA, mm, m, 1, r->JV, mm, m, 1, r->JT, mm, m, 1, m, m, m, INT_MAX, c},
                    2 * c, st));
  FIRAL_CHECK(bgemm(BGemm{r->JV, mm, 1, m, r->JT, mm, m, 1, r->JA, mm, m, 1, m, m, m, c, INT_MAX},
                    2 * c, st));
  FIRAL_CHECK(jacobi_launch(r->JA, r->JV, r->lam, m, d, c, c, 1, st));
  k_round_nu<<<1, 1024, 0, st>>>(r->lam, m, d, c, r->eta, r->nu + t + 1);
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
  RREQ(x->c <= 30000, "firal_round_create: c = %d above the Round step's limit 30000", x->c);
  RREQ((flags & ~FIRAL_ROUND_FP32) == 0, "firal_round_create: unknown flags 0x%x", flags);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(x->device));
  Round* r = new Round();
  r->x = x;
  r->d = x->d;
  r->c = x->c;
  r->m = x->d + (x->d & 1);
  r->ldw = (int)cdiv(x->d, 16) * 16;
  r->b = b;
  r->t = 0;
  r->n_pool = x->n_pool;
  r->N = x->N;
  r->eta = eta;
  r->fp32 = (flags & FIRAL_ROUND_FP32) != 0;
  const int d = r->d, c = r->c, m = r->m;
  // rows per scoring chunk: the class-term buffer c x R stays within 1 GiB
  const int64_t cap = std::max<int64_t>(256, (((int64_t)1 << 27) / c) / 256 * 256);
  r->R = std::min<int64_t>(cdiv(r->n_pool, 256) * 256, cap);
  r->nparts = cdiv(r->n_pool, 256);
  std::vector<int32_t> tiles;
  syrk_plan(FIRAL_F64, d, c, &tiles, &r->splits);
  r->ntiles = (int)(tiles.size() / 2);
  const int64_t dd = (int64_t)d * d, mm = (int64_t)m * m;
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
  RALLOC(r->JA, sizeof(double) * 2 * c * mm);
  RALLOC(r->JV, sizeof(double) * c * mm);
  RALLOC(r->JT, sizeof(double) * 2 * c * mm);
  RALLOC(r->lam, sizeof(double) * 2 * c * m);
  RALLOC(r->W, sizeof(double) * c * d * r->ldw);
  RALLOC(r->wts, sizeof(double) * c * r->ldw * 2);
  RALLOC(r->Tb, sizeof(double) * c * r->R);
  RALLOC(r->pval, sizeof(double) * r->nparts);
  RALLOC(r->pidx, sizeof(int64_t) * r->nparts);
  RALLOC(r->nu, sizeof(double) * (b + 1));
  RALLOC(r->smax, sizeof(double) * b);
  RALLOC(r->sel, sizeof(int64_t) * b);
  RALLOC(r->mask, sizeof(int32_t) * r->n_pool);
  RALLOC(r->flags, sizeof(int32_t) * 2);
  RALLOC(r->crit, sizeof(double));
  RALLOC(r->gpart, sizeof(double) * r->splits * c * dd);
  RALLOC(r->tiles, sizeof(int32_t) * tiles.size());
  if (r->fp32) {
    RALLOC(r->Wf, sizeof(float) * c * d * r->ldw);
    RALLOC(r->wtsf, sizeof(float) * c * r->ldw * 2);
  }
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
#define RCHK(e)                 \
  do {                          \
    int rc_ = (e);              \
    if (rc_ < 0) return fail(rc_); \
  } while (0)
  RCHK(fill_i32(r->flags, 1, INT_MAX, st));
  RCHK(fill_i32(r->flags + 1, 1, 0, st));
  RCHK(fill_i32(r->mask, r->n_pool, 0, st));
  RCHK(fill(r->Cm, c * dd, 0.0, st));
  RCHK(fill(r->Hacc, c * dd, 0.0, st));
  RCHK(fill(r->W, (int64_t)c * d * r->ldw, 0.0, st));
  k_fill_i64<<<(unsigned)cdiv(b, 256), 256, 0, st>>>(r->sel, b, -1);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(fill(r->nu, 1, std::sqrt((double)d * c), st));
  // Sigma_o blocks (rows weighted by [z ; 1], plus lambda I), factorised
  k_round_omega<<<(unsigned)cdiv(r->N, 256), 256, 0, st>>>(z, r->n_pool, r->N, r->omega);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(gram64_launch(x->prec, x->X, x->H, r->omega, r->N, d, c, r->tiles, r->ntiles, r->splits,
                     lambda, r->gpart, r->Lf, st));
  RCHK(chol_blocks_launch(r->Lf, r->JA, d, c, r->flags, st));
  // H_o blocks: the labeled rows with unit weight
  const size_t es = x->prec == FIRAL_F64 ? 8 : 4;
  RCHK(gram64_launch(x->prec, (const char*)x->X + es * r->n_pool * d,
                     (const char*)x->H + es * r->n_pool * c, nullptr, r->N - r->n_pool, d, c,
                     r->tiles, r->ntiles, r->splits, 0.0, r->gpart, r->Ho, st));
  k_tri_inv<<<c, 256, 0, st>>>(r->Lf, r->Li, d);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  // O_k = L^-1 H_o L^-T (JV as the intermediate H_o L^-T)
  RCHK(bgemm(BGemm{r->Ho, dd, d, 1, r->Li, dd, 1, d, r->JV, dd, d, 1, d, d, d, INT_MAX, INT_MAX},
             c, st));
  RCHK(bgemm(BGemm{r->Li, dd, d, 1, r->JV, dd, d, 1, r->Ot, dd, d, 1, d, d, d, INT_MAX, INT_MAX},
             c, st));
  // round 1: E = O / b, eigenpairs, nu_1 = sqrt(dc), W and weights
  k_pad_comb<<<(unsigned)cdiv((int64_t)c * mm, 256), 256, 0, st>>>(
      r->Ot, 1.0 / b, nullptr, 0.0, r->JA + (int64_t)c * mm, d, m, c);
  if (hipGetLastError() != hipSuccess) return fail(FIRAL_EHIP);
  RCHK(jacobi_launch(r->JA + (int64_t)c * mm, r->JV, r->lam + (int64_t)c * m, m, d, 0, c, 0, st));
  RCHK(round_operand(r, r->nu, st));
  int32_t bad = INT_MAX;
  if (hipMemcpyAsync(&bad, r->flags, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    set_error("firal_round_create: set-up failed");
    return fail(FIRAL_EHIP);
  }
  if (bad != INT_MAX) {
    set_error("Sigma block %d of the Round step is not positive definite", bad);
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
  int32_t err = 0;
  FIRAL_HIP(hipMemcpyAsync(&err, r->flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (selected && n > 0)
    FIRAL_HIP(hipMemcpyAsync(selected, r->sel, sizeof(int64_t) * n, hipMemcpyDeviceToHost, st));
  if (nu) FIRAL_HIP(hipMemcpyAsync(nu, r->nu, sizeof(double) * (n + 1), hipMemcpyDeviceToHost, st));
  if (score_max && n > 0)
    FIRAL_HIP(hipMemcpyAsync(score_max, r->smax, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  FIRAL_HIP(hipStreamSynchronize(st));
  if (t) *t = n;
  if (err) {
    set_error("Round step: no unselected pool row with a finite score was left");
    return FIRAL_EINVAL;
  }
  return FIRAL_OK;
}

extern "C" int firal_round_criterion(firal_round round, double* out, void* stream) {
  RREQ(round != nullptr && out != nullptr, "firal_round_criterion: null argument");
  Round* r = reinterpret_cast<Round*>(round);
  hipStream_t st = (hipStream_t)stream;
  FIRAL_HIP(hipSetDevice(r->x->device));
  const int d = r->d, c = r->c, m = r->m;
  k_pad_comb<<<(unsigned)cdiv((int64_t)c * m * m, 256), 256, 0, st>>>(r->Hacc, 1.0, nullptr, 0.0,
                                                                      r->JA, d, m, c);
  FIRAL_LAUNCHED();
  FIRAL_CHECK(jacobi_launch(r->JA, nullptr, r->lam, m, d, c, 0, 0, st));
  k_min_eig<<<1, 1024, 0, st>>>(r->lam, m, d, c, r->crit);
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
